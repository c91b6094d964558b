// Binning and ordering on gfx950 (Alg. 1: DuplicateWithKeys, SortByKeys,
// IdentifyTileRanges).
//
// Design: the per-view depth order is established once over the N Gaussians
// (LSD radix sort of the float32 depth bits, stable, so equal depths keep
// ascending id).  Binning is then two-level: every depth-ordered Gaussian emits
// one coarse entry per super-tile (S x S tiles) its square touches, keyed by
// the super-tile and carrying the mask of the super-tile's tiles it reaches; a
// stable sort of the coarse entries by super-tile keeps depth order inside each
// super-tile's list.  A tile's list is the sub-sequence of its super-tile's
// list whose mask holds the tile, which the blending kernels compact on the fly
// (64-lane ballot + prefix, walk.hpp): exactly the tile's (depth bits,
// id)-ordered set of overlapping splats - the order a global (tile, depth, id)
// sort gives - without sorting or storing (Gaussian, tile) pairs at all.
//
// When a batched call repeats a camera at several times, the 3D Gaussians are
// sorted and binned once per camera (a static group) onto a super-tile grid of
// the group's own, and each view bins only its 4D Gaussians; the blending
// kernels merge the two lists by depth.
//
// Every LSD pass is: per-block digit histogram -> per-digit scan across blocks
// -> stable scatter.  The stable scatter ranks keys inside a wave with ballots
// (64-lane match on the digit bits), orders the block's tile in LDS and writes
// coalesced runs per digit.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

__device__ __forceinline__ uint64_t read_count(const unsigned long long* dc, uint64_t hc) {
    return dc ? (uint64_t)(*dc) : hc;
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
}

// inclusive-to-exclusive block scan of one value per thread (256 threads)
template <typename T>
__device__ inline T block_exclusive_scan_256(T v, T* s_buf, T& total) {
    // wave scans, then the four wave totals (s_buf[0..3])
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    T incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_buf[w] = incl;
    __syncthreads();
    T base = (T)0;
    for (int k = 0; k < w; ++k) base += s_buf[k];
    total = s_buf[0] + s_buf[1] + s_buf[2] + s_buf[3];
    __syncthreads();  // s_buf is free again for the caller
    return base + incl - v;
}

// ---------------------------------------------------------------------------
// Radix sort pass (up to 11 bits per pass)
// ---------------------------------------------------------------------------
// In-place exclusive scan of s[0 .. radix) (radix <= 2^MB) by the block's 256
// threads, each owning 2^MB / 256 consecutive digits; returns the total.
template <int MB>
__device__ inline uint32_t block_scan_digits(uint32_t* s, int radix, uint32_t* s_buf) {
    constexpr int DPT = (1 << MB) / kSortThreads;
    const int d0 = threadIdx.x * DPT;
    uint32_t v[DPT];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        v[q] = d0 + q < radix ? s[d0 + q] : 0u;
        sum += v[q];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan_256<uint32_t>(sum, s_buf, total);
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
        if (d0 + q < radix) s[d0 + q] = run;
        run += v[q];
    }
    __syncthreads();
    return total;
}

// MB: largest digit width the instantiation handles (LDS is sized for it).
// skip_empty: keys whose upper 16 bits are zero (coarse entries with an empty
// tile mask) are left out of the counts (and, in the downsweep, of the output).
template <int MB, int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_radix_upsweep(const uint32_t* __restrict__ keys,
                                                                const unsigned long long* dcount, uint64_t hcount,
                                                                int shift, int nbits, uint32_t* __restrict__ hist,
                                                                int nblocks, uint64_t seg_stride, int skip_empty) {
    __shared__ uint32_t s_hist[4][1 << MB];
    const int radix = 1 << nbits;
    keys += (size_t)blockIdx.y * seg_stride;
    hist += (size_t)blockIdx.y * radix * nblocks;
    const uint32_t mask = (uint32_t)radix - 1u;
    const int tid = threadIdx.x, w = tid >> 6;
    const uint64_t n = read_count(dcount, hcount);
    const uint64_t begin = (uint64_t)blockIdx.x * (kSortThreads * ITEMS);
    if (begin >= n) return;  // blocks past the live count are never scanned (uniform)
    for (int d = tid; d < 4 * radix; d += kSortThreads) s_hist[d / radix][d % radix] = 0;
    __syncthreads();
    for (int k = 0; k < ITEMS; ++k) {
        const uint64_t idx = begin + (uint64_t)k * kSortThreads + tid;
        if (idx < n) {
            const uint32_t key = keys[idx];
            if (!skip_empty || (key >> 16) != 0u) atomicAdd(&s_hist[w][(key >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < radix; d += kSortThreads)
        hist[(size_t)d * nblocks + blockIdx.x] = s_hist[0][d] + s_hist[1][d] + s_hist[2][d] + s_hist[3][d];
}

// one block per (digit, segment): exclusive scan of that digit's per-block
// counts over the blocks that hold live keys (4 counts per thread per round)
__global__ void __launch_bounds__(256) k_radix_digit_scan(uint32_t* __restrict__ hist, int nblocks, int radix,
                                                          uint32_t* __restrict__ totals,
                                                          const unsigned long long* dcount, uint64_t hcount,
                                                          int tile) {
    __shared__ uint32_t s_buf[256];
    const uint64_t n = read_count(dcount, hcount);
    const int live = (int)min((uint64_t)nblocks, (n + tile - 1) / tile);
    uint32_t* h = hist + (size_t)blockIdx.y * radix * nblocks + (size_t)blockIdx.x * nblocks;
    totals += (size_t)blockIdx.y * radix;
    uint32_t carry = 0;
    for (int start = 0; start < live; start += 1024) {
        const int i0 = start + 4 * (int)threadIdx.x;
        uint32_t v[4];
        uint32_t sum = 0;
        for (int q = 0; q < 4; ++q) {
            v[q] = i0 + q < live ? h[i0 + q] : 0u;
            sum += v[q];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive_scan_256<uint32_t>(sum, s_buf, tot) + carry;
        for (int q = 0; q < 4; ++q) {
            if (i0 + q < live) h[i0 + q] = ex;
            ex += v[q];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int MB, int ITEMS>
__global__ void __launch_bounds__(kSortThreads) k_radix_downsweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const unsigned long long* dcount, uint64_t hcount, int shift, int nbits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int nblocks,
    const unsigned long long* out_offset, uint64_t seg_stride, int64_t* __restrict__ digit_ranges, int n_digit_ranges,
    const uint32_t* __restrict__ val_map, int skip_empty, unsigned long long* out_count) {
    __shared__ uint32_t s_wcount[4][1 << MB];
    __shared__ uint32_t s_dstart[1 << MB];
    __shared__ uint32_t s_gbase[1 << MB];
    __shared__ uint32_t s_buf[256];
    constexpr int TILE = kSortThreads * ITEMS;
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];

    const uint64_t n = read_count(dcount, hcount);
    const uint64_t begin = (uint64_t)blockIdx.x * TILE;
    if (begin >= n) {  // uniform over the block
        // no keys at all: the kept count is still written (block 0 holds keys otherwise)
        if (out_count && n == 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *out_count = 0ull;
        return;
    }
    const int radix = 1 << nbits;
    {
        const size_t so = (size_t)blockIdx.y * seg_stride;
        keys_in += so; vals_in += so; keys_out += so; vals_out += so;
        hist += (size_t)blockIdx.y * radix * nblocks;
        totals += (size_t)blockIdx.y * radix;
    }
    const uint32_t mask = (uint32_t)radix - 1u;
    const int tid = threadIdx.x, w = tid >> 6, lane = __lane_id();

    for (int d = tid; d < 4 * radix; d += kSortThreads) s_wcount[d / radix][d % radix] = 0;
    // global base of digit d = (exclusive scan of totals)[d] + this block's scanned count
    for (int d = tid; d < radix; d += kSortThreads) s_gbase[d] = totals[d];
    __syncthreads();
    const uint32_t n_out = block_scan_digits<MB>(s_gbase, radix, s_buf);
    if (out_count && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *out_count = n_out;
    const unsigned long long off = out_offset ? *out_offset : 0ull;
    // a single-pass sort over whole keys: the digit runs are the key ranges
    if (digit_ranges && blockIdx.x == 0 && blockIdx.y == 0)
        for (int d = tid; d < n_digit_ranges; d += kSortThreads) {
            digit_ranges[2 * (size_t)d] = (int64_t)off + s_gbase[d];
            digit_ranges[2 * (size_t)d + 1] = (int64_t)off + s_gbase[d] + totals[d];
        }
    for (int d = tid; d < radix; d += kSortThreads) s_gbase[d] += hist[(size_t)d * nblocks + blockIdx.x];

    // wave w owns items [begin + w * 64 ITEMS, begin + (w + 1) * 64 ITEMS), ITEMS rounds of 64
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
    const unsigned long long lt = lanemask_lt();
    for (int r = 0; r < ITEMS; ++r) {
        const uint64_t idx = begin + (uint64_t)w * (ITEMS * 64) + (uint64_t)r * 64 + lane;
        key[r] = idx < n ? keys_in[idx] : 0u;
        const bool valid = idx < n && (!skip_empty || (key[r] >> 16) != 0u);
        val[r] = valid ? vals_in[idx] : 0u;
        const uint32_t d = (key[r] >> shift) & mask;
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        uint32_t base = 0;
        if (valid) base = s_wcount[w][d];
        rank[r] = base + before;
        if (valid && before == 0) s_wcount[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: prefix over waves, block total per digit, then start of each
    // digit's run in the block-sorted tile
    for (int d = tid; d < radix; d += kSortThreads) {
        uint32_t run = 0;
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = s_wcount[q][d];
            s_wcount[q][d] = run;
            run += c;
        }
        s_dstart[d] = run;
    }
    __syncthreads();
    const int cnt = (int)block_scan_digits<MB>(s_dstart, radix, s_buf);  // keys this block places
    for (int r = 0; r < ITEMS; ++r) {
        const uint64_t idx = begin + (uint64_t)w * (ITEMS * 64) + (uint64_t)r * 64 + lane;
        if (idx < n && (!skip_empty || (key[r] >> 16) != 0u)) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t pos = s_dstart[d] + s_wcount[w][d] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();
    for (int p = tid; p < cnt; p += kSortThreads) {
        const uint32_t k = s_keys[p];
        const uint32_t d = (k >> shift) & mask;
        const uint64_t dst = off + (uint64_t)s_gbase[d] + (uint64_t)(p - (int)s_dstart[d]);
        keys_out[dst] = k;
        vals_out[dst] = val_map ? val_map[s_vals[p]] : s_vals[p];
    }
}

int radix_blocks(uint64_t capacity, int items) {
    const uint64_t tile = (uint64_t)kSortThreads * items;
    return (int)((capacity + tile - 1) / tile);
}
size_t radix_hist_words(uint64_t capacity, int n_seg, int max_bits, int items) {
    return ((size_t)1 << max_bits) * (size_t)std::max(1, radix_blocks(capacity, items)) * (size_t)std::max(1, n_seg);
}

bool radix_pass_fits(uint64_t capacity, int n_seg, int nbits, int items, size_t hist_words, size_t totals_words) {
    if (nbits < 1 || nbits > kMaxRadixBits || n_seg < 0 || (items != 2 && items != kSortItems)) return false;
    if (items == 2 && nbits > 8) return false;
    return radix_hist_words(capacity, n_seg, nbits, items) <= hist_words &&
           ((size_t)1 << nbits) * (size_t)std::max(1, n_seg) <= totals_words;
}

bool launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                       const unsigned long long* dcount, uint64_t hcount, uint64_t capacity, int shift, int nbits,
                       uint32_t* hist, size_t hist_words, uint32_t* totals, size_t totals_words,
                       const unsigned long long* out_offset, hipStream_t st, int n_seg, uint64_t seg_stride,
                       int64_t* digit_ranges, int n_digit_ranges, int items, const uint32_t* val_map, int skip_empty,
                       unsigned long long* out_count) {
    // every block writes 2^nbits counts per segment: refuse a pass whose
    // histogram or digit totals would not fit the buffers it was given
    if (!radix_pass_fits(capacity, n_seg, nbits, items, hist_words, totals_words)) return false;
    const int nb = radix_blocks(capacity, items);
    if (nb == 0 || n_seg == 0) return true;
    const dim3 grid(nb, n_seg);
    // the smallest instantiation that holds the digit (LDS is sized by it)
#define H4D_RADIX_PASS(MB, IT)                                                                                       \
    do {                                                                                                              \
        k_radix_upsweep<MB, IT><<<grid, kSortThreads, 0, st>>>(keys_in, dcount, hcount, shift, nbits, hist, nb,       \
                                                              seg_stride, skip_empty);                               \
        k_radix_digit_scan<<<dim3(1 << nbits, n_seg), 256, 0, st>>>(hist, nb, 1 << nbits, totals, dcount, hcount,    \
                                                                    kSortThreads * IT);                              \
        k_radix_downsweep<MB, IT><<<grid, kSortThreads, 0, st>>>(keys_in, vals_in, keys_out, vals_out, dcount,        \
                                                                hcount, shift, nbits, hist, totals, nb, out_offset,   \
                                                                seg_stride, digit_ranges, n_digit_ranges, val_map,    \
                                                                skip_empty, out_count);                               \
    } while (0)
    if (items == 2 && nbits <= 8) {
        H4D_RADIX_PASS(8, 2);  // short key sets: more, smaller blocks
    } else {  // (a grid sized for smaller blocks only adds blocks past the live count)
        if (nbits <= 8) H4D_RADIX_PASS(8, kSortItems);
        else if (nbits == 9) H4D_RADIX_PASS(9, kSortItems);
        else if (nbits == 10) H4D_RADIX_PASS(10, kSortItems);
        else H4D_RADIX_PASS(kMaxRadixBits, kSortItems);
    }
#undef H4D_RADIX_PASS
    return true;
}

// ---------------------------------------------------------------------------
// 64-bit exclusive scan of (optionally gathered) 32-bit counts.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx,
                                                     int n, unsigned long long* __restrict__ partials) {
    __shared__ unsigned long long s_buf[256];
    const int begin = blockIdx.x * kScanTile + threadIdx.x * 8;
    unsigned long long s = 0;
    for (int k = 0; k < 8; ++k) {
        const int i = begin + k;
        if (i < n) s += in[idx ? idx[i] : i];
    }
    unsigned long long tot;
    block_exclusive_scan_256<unsigned long long>(s, s_buf, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_top(unsigned long long* __restrict__ partials, int nparts) {
    __shared__ unsigned long long s_buf[256];
    unsigned long long carry = 0;
    for (int start = 0; start < nparts; start += 256) {
        const int i = start + threadIdx.x;
        const unsigned long long v = i < nparts ? partials[i] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_exclusive_scan_256<unsigned long long>(v, s_buf, tot);
        if (i < nparts) partials[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) partials[nparts] = carry;
}

// With run_start: for every run of 256 outputs, the index whose range
// [out[i], out[i + 1]) holds the run's first output (runs below run_cap).
__global__ void __launch_bounds__(256) k_scan_down(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx,
                                                   int n, const unsigned long long* __restrict__ partials, int nparts,
                                                   unsigned long long* __restrict__ out,
                                                   uint32_t* __restrict__ run_start, uint64_t run_cap) {
    __shared__ unsigned long long s_buf[256];
    const int begin = blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t v[8];
    unsigned long long s = 0;
    for (int k = 0; k < 8; ++k) {
        const int i = begin + k;
        v[k] = i < n ? in[idx ? idx[i] : i] : 0u;
        s += v[k];
    }
    unsigned long long tot;
    unsigned long long run = block_exclusive_scan_256<unsigned long long>(s, s_buf, tot) + partials[blockIdx.x];
    for (int k = 0; k < 8; ++k) {
        const int i = begin + k;
        if (i < n) {
            out[i] = run;
            if (run_start)
                for (uint64_t r = (run + 255) / 256; r * 256 < run + v[k] && r < run_cap; ++r) run_start[r] = (uint32_t)i;
        }
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partials[nparts];
}

int scan_blocks(int n) { return (n + kScanTile - 1) / kScanTile; }

void launch_scan_u32_u64(const uint32_t* in, const uint32_t* idx, int n, unsigned long long* out,
                         unsigned long long* partials, hipStream_t st, uint32_t* run_start, uint64_t run_cap) {
    const int nb = std::max(1, scan_blocks(n));
    k_scan_reduce<<<nb, 256, 0, st>>>(in, idx, n, partials);
    k_scan_top<<<1, 256, 0, st>>>(partials, nb);
    k_scan_down<<<nb, 256, 0, st>>>(in, idx, n, partials, nb, out, run_start, run_cap);
}

// ---------------------------------------------------------------------------
// Two-level binning.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t pack_rect(uint32_t x0, uint32_t x1, uint32_t y0, uint32_t y1) {
    return (uint64_t)x0 | ((uint64_t)x1 << 16) | ((uint64_t)y0 << 32) | ((uint64_t)y1 << 48);
}

// Margin (log2 units) between the FP64 tile test and the FP32 per-pixel test:
// the FP32 exponent of a pixel is within about 1e-5 of its exact value, so a
// tile none of whose pixel centres reaches alpha = 1/255 * 2^-margin in exact
// arithmetic has no pixel that the blending kernels would blend.
constexpr double kCullMargin = 1e-3;

// The alpha >= 1/255 region of one splat as the tile test needs it:
// -p2 = a dx^2 - b dx dy + c dy^2 <= t, with dx, dy offsets from the centre.
// Set up in FP64 per splat; the per-row test runs in FP32 on intervals widened
// by pad_x / pad_y: 2e-3 of the ellipse's half-extent plus 0.01 px, several
// times the FP32 rounding of the extent (whose worst case, near the ellipse's
// top and bottom, is about 5e-4 of the half-width).

__host__ __device__ inline CullShape cull_shape(const Rec& rec) {
    CullShape cs;
    const double a = -(double)rec.a.z, b = rec.a.w, c = -(double)rec.b.x, op = rec.b.y;
    cs.ui = rec.c.y; cs.uf = rec.a.x; cs.vi = rec.c.z; cs.vf = rec.a.y;
    cs.px0 = (int)(rec.d.x & 0xFFFFu); cs.px1 = (int)(rec.d.x >> 16);
    cs.py0 = (int)(rec.d.y & 0xFFFFu); cs.py1 = (int)(rec.d.y >> 16);
    const double det4 = 4.0 * a * c - b * b;
    cs.mode = 0;
    cs.b = cs.inv2a = cs.four_at = cs.det4 = cs.y_full = cs.y_ext = cs.pad_x = cs.pad_y = 0.f;
    // a proper ellipse only; otherwise keep every overlapped tile
    if (a > 0.0 && c > 0.0 && det4 > 1e-12 * 4.0 * a * c && op > 0.0) {
        const double t = log2(255.0 * op) + kCullMargin;
        if (t <= 0.0) {
            cs.mode = 2;
        } else {
            cs.mode = 1;
            const double y_full = sqrt(4.0 * a * t / det4), x_ext = sqrt(4.0 * c * t / det4);
            cs.b = (float)b;
            cs.inv2a = (float)(0.5 / a);
            cs.four_at = (float)(4.0 * a * t);
            cs.det4 = (float)det4;
            cs.y_full = (float)y_full;
            cs.y_ext = (float)(b * x_ext / (2.0 * c));
            cs.pad_y = (float)(2e-3 * y_full + 1e-2);
            cs.pad_x = (float)(2e-3 * (x_ext + fabs(b) * y_full * 0.5 / a) + 1e-2);
        }
    }
    return cs;
}

// Pixel-centre offsets from the splat's centre (x: ui + uf, y: vi + vf) of
// the first and last pixel column of tile column tx, and of the first and last
// pixel row of tile row ty, inside its pixel square.
template <int TILE>
__host__ __device__ __forceinline__ float col_x0(const CullShape& cs, int tx) {
    return ((float)max(tx * TILE, cs.px0) + 0.5f - cs.ui) - cs.uf;
}
template <int TILE>
__host__ __device__ __forceinline__ float col_x1(const CullShape& cs, int tx) {
    return ((float)min(tx * TILE + TILE - 1, cs.px1) + 0.5f - cs.ui) - cs.uf;
}
template <int TILE>
__host__ __device__ __forceinline__ float row_y0(const CullShape& cs, int ty) {
    return ((float)max(ty * TILE, cs.py0) + 0.5f - cs.vi) - cs.vf;
}
template <int TILE>
__host__ __device__ __forceinline__ float row_y1(const CullShape& cs, int ty) {
    return ((float)min(ty * TILE + TILE - 1, cs.py1) + 0.5f - cs.vi) - cs.vf;
}
// Whether tile row ty's slab of pixel-centre offsets meets the ellipse's
// height (widened by pad_y).
template <int TILE>
__host__ __device__ __forceinline__ bool row_meets(const CullShape& cs, int ty) {
    return !(row_y1<TILE>(cs, ty) < -cs.y_full - cs.pad_y || row_y0<TILE>(cs, ty) > cs.y_full + cs.pad_y);
}
// The ellipse's x-extent [xl, xr] over tile row ty's slab (from its leftmost
// and rightmost points clamped into the slab), widened by pad_x.
template <int TILE>
__host__ __device__ __forceinline__ void row_extent(const CullShape& cs, int ty, float& xl, float& xr) {
    const float Y0 = row_y0<TILE>(cs, ty), Y1 = row_y1<TILE>(cs, ty);
    const float yr = fminf(fmaxf(cs.y_ext, Y0), Y1), yl = fminf(fmaxf(-cs.y_ext, Y0), Y1);
    xr = (cs.b * yr + sqrtf(fmaxf(0.f, cs.four_at - yr * yr * cs.det4))) * cs.inv2a + cs.pad_x;
    xl = (cs.b * yl - sqrtf(fmaxf(0.f, cs.four_at - yl * yl * cs.det4))) * cs.inv2a - cs.pad_x;
}

// Tiles (bit ly * S + lx) of the super-tile at tile origin (bx, by) that the
// splat's tile rectangle [tx0, tx1] x [ty0, ty1] overlaps and, when cull is
// set, in which the ellipse's x-extent over the tile row's slab meets the
// tile's pixel-centre x-range (the test of row_span, per entry: splats taller
// than the span table).
template <int TILE>
__host__ __device__ inline uint32_t tile_mask(const CullShape& cs, bool cull, uint32_t tx0, uint32_t tx1, uint32_t ty0,
                                     uint32_t ty1, uint32_t bx, uint32_t by) {
    constexpr uint32_t S = (uint32_t)super_factor(TILE);
    const uint32_t lx0 = max(tx0, bx) - bx, lx1 = min(tx1, bx + S - 1u) - bx;
    const uint32_t ly0 = max(ty0, by) - by, ly1 = min(ty1, by + S - 1u) - by;
    uint32_t cols = 0u, rows = 0u;  // bit l: column / row l overlaps the rectangle
#pragma unroll
    for (uint32_t l = 0; l < S; ++l) {
        cols |= (l >= lx0 && l <= lx1) ? 1u << l : 0u;
        rows |= (l >= ly0 && l <= ly1) ? 1u << l : 0u;
    }
    if (!cull) {
        uint32_t mask = 0u;
#pragma unroll
        for (uint32_t ly = 0; ly < S; ++ly)
            if ((rows >> ly) & 1u) mask |= cols << (ly * S);
        return mask;
    }
    // the columns' pixel-centre offset intervals do not depend on the row
    float X0[S], X1[S];
#pragma unroll
    for (uint32_t lx = 0; lx < S; ++lx) {
        X0[lx] = col_x0<TILE>(cs, (int)(bx + lx));
        X1[lx] = col_x1<TILE>(cs, (int)(bx + lx));
    }
    uint32_t mask = 0u;
#pragma unroll
    for (uint32_t ly = 0; ly < S; ++ly) {
        if (!((rows >> ly) & 1u)) continue;
        const int ty = (int)(by + ly);
        if (!row_meets<TILE>(cs, ty)) continue;
        float xl, xr;
        row_extent<TILE>(cs, ty, xl, xr);
#pragma unroll
        for (uint32_t lx = 0; lx < S; ++lx)
            if (((cols >> lx) & 1u) && X1[lx] >= xl && X0[lx] <= xr) mask |= 1u << (ly * S + lx);
    }
    return mask;
}

// The tile columns of tile row ty that the test above keeps, as one word:
// first column | (last + 1) << 16 (0: none).  The columns whose x-range meets
// [xl, xr] form one run (both ends of a column's range grow with the column):
// a first guess from the pixel coordinates, then stepped to the exact ends of
// the same comparisons.
template <int TILE>
__host__ __device__ inline uint32_t row_span(const CullShape& cs, int ty, int tx0, int tx1) {
    if (!row_meets<TILE>(cs, ty)) return 0u;
    float xl, xr;
    row_extent<TILE>(cs, ty, xl, xr);
    const float lo = (float)(tx0 - 1), hi = (float)(tx1 + 1);
    int cl = (int)fminf(fmaxf(ceilf((xl + cs.ui + cs.uf + 0.5f) * (1.f / TILE)) - 1.f, lo), hi);
    cl = min(max(cl, tx0), tx1 + 1);
    while (cl > tx0 && col_x1<TILE>(cs, cl - 1) >= xl) --cl;
    while (cl <= tx1 && !(col_x1<TILE>(cs, cl) >= xl)) ++cl;
    int cr = (int)fminf(fmaxf(floorf((xr + cs.ui + cs.uf - 0.5f) * (1.f / TILE)), lo), hi);
    cr = min(max(cr, tx0 - 1), tx1);
    while (cr < tx1 && col_x0<TILE>(cs, cr + 1) <= xr) ++cr;
    while (cr >= tx0 && !(col_x0<TILE>(cs, cr) <= xr)) --cr;
    return cl <= cr ? (uint32_t)cl | ((uint32_t)(cr + 1) << 16) : 0u;
}

// Flags in the top bits of a splat's packed tile rectangle (tile coordinates
// stay below 2^14): the shape test per coarse entry, or no test at all.
constexpr uint64_t kRectShape = 1ull << 63, kRectFull = 1ull << 62;
constexpr uint64_t kRectCoords = ~(kRectShape | kRectFull);

// Where depth-ordered entry j of a pass (segment layout sg) belongs: the view
// whose records hold it and, for its super-tile keys, that view's grid and the
// grid's first super-tile id relative to the pass (a static group's grid for
// the group segments).
struct SegPos {
    int view, super0;
};
__device__ __forceinline__ SegPos seg_of(int j, const SegLayout& sg, const ViewParams* __restrict__ views, int v0) {
    const int split = sg.na * sg.la;
    if (j < split) {
        const int v = v0 + j / sg.la;
        return SegPos{v, views[v].super_base - views[v0].super_base};
    }
    const int leader = views[(j - split) / sg.lb].group_leader;
    return SegPos{leader, views[leader].static_super_base - views[v0].super_base};
}

// First index i in [lo, hi] with pred(i) (hi + 1 if none), for a predicate
// that is false up to some index and true from there on, starting from a
// guess; and the last index with pred (lo - 1 if none) for one that is true up
// to some index and false after it.
template <typename P>
__host__ __device__ inline int first_true(float guess, int lo, int hi, P pred) {
    int i = (int)fminf(fmaxf(guess, (float)lo), (float)(hi + 1));
    while (i > lo && pred(i - 1)) --i;
    while (i <= hi && !pred(i)) ++i;
    return i;
}
template <typename P>
__host__ __device__ inline int last_true(float guess, int lo, int hi, P pred) {
    int i = (int)fminf(fmaxf(guess, (float)(lo - 1)), (float)hi);
    while (i < hi && pred(i + 1)) ++i;
    while (i >= lo && !pred(i)) --i;
    return i;
}

// The tile rows [r0, r1] of [ty0, ty1] whose slab meets the ellipse (a run:
// both ends of a row's slab grow with the row; r1 < r0 when none).
template <int TILE>
__host__ __device__ inline void slab_rows(const CullShape& cs, int ty0, int ty1, int& r0, int& r1) {
    const float h = cs.y_full + cs.pad_y, cy = cs.vi + cs.vf;
    r0 = first_true(ceilf((cy - h + 0.5f) * (1.f / TILE)) - 1.f, ty0, ty1,
                    [&](int ty) { return !(row_y1<TILE>(cs, ty) < -h); });
    r1 = last_true(floorf((cy + h - 0.5f) * (1.f / TILE)), r0, ty1,
                   [&](int ty) { return !(row_y0<TILE>(cs, ty) > h); });
}

// Tiles of the super-tile at tile origin (bx, by) in the tabulated spans of
// rows [ty0, ty1] (span_row[row - ty0]), as tile_mask's bits.
template <int TILE>
__host__ __device__ inline uint32_t span_mask(const uint32_t* span_row, uint32_t ty0, uint32_t ty1, uint32_t bx,
                                              uint32_t by) {
    constexpr uint32_t S = (uint32_t)super_factor(TILE);
    uint32_t m = 0u;
#pragma unroll
    for (uint32_t ly = 0; ly < S; ++ly) {
        const uint32_t ty = by + ly;
        if (ty < ty0 || ty > ty1) continue;
        const uint32_t e = span_row[ty - ty0];
        const uint32_t lo = (e & 0xFFFFu) > bx ? (e & 0xFFFFu) : bx, hi = (e >> 16) < bx + S ? (e >> 16) : bx + S;
        if (lo < hi) m |= ((1u << (hi - bx)) - (1u << (lo - bx))) << (ly * S);
    }
    return m;
}

// Per depth-ordered entry j of the pass: its tile rectangle and its
// super-tile count.  With culling (shapes != null) the rectangle shrinks to
// the rows whose slab meets the ellipse and to the columns any of their spans
// keeps (the tiles tile_mask can keep; a splat with none emits nothing), and
// the spans of up to kSpanRows rows are tabulated for the emission
// (spans[j * kSpanRows + row - first row]); a taller splat keeps its shape
// (kRectShape: tested per entry) and one without a proper ellipse its square
// (kRectFull: untested).  The spans of a wave's splats are computed one
// (splat, row) per lane: a wave's rows are numbered by a prefix sum over its
// lanes, and each round of 64 finds its rows' splats by a max-scan of the
// lanes' first rows.
// One entry per thread; each workgroup also leaves its sum of counts for
// the offsets' scan (partials[blockIdx.x]).
template <int TILE>
__global__ void __launch_bounds__(256, 6) k_coarse_count(const uint32_t* __restrict__ sorted_gid, int n, int N,
                                                      SegLayout sg, const Rec* __restrict__ recs,
                                                      const ViewParams* __restrict__ views, int v0,
                                                      uint32_t* __restrict__ cnt, uint64_t* __restrict__ rect_sorted,
                                                      CullShape* __restrict__ shapes, uint32_t* __restrict__ spans,
                                                      unsigned long long* __restrict__ partials) {
    constexpr uint32_t S = (uint32_t)super_factor(TILE);
    __shared__ unsigned long long s_buf[256];
    __shared__ CullShape s_cs[256];
    __shared__ int s_cmin[256], s_cmax[256];
    __shared__ int s_slot[4][64];
    const int tid = (int)threadIdx.x, lane = __lane_id(), w = tid >> 6;
    const int j = blockIdx.x * 256 + tid;
    bool keep = false;
    uint64_t flags = 0ull;
    int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1, r0 = 0, nrows = 0;
    if (j < n) {
        const SegPos sp = seg_of(j, sg, views, v0);
        const Rec& rec = recs[(size_t)sp.view * N + sorted_gid[j]];
        const uint4 d = rec.d;
        if (d.w != 0u) {
            keep = true;
            tx0 = (int)((d.x & 0xFFFFu) / TILE); tx1 = (int)((d.x >> 16) / TILE);
            ty0 = (int)((d.y & 0xFFFFu) / TILE); ty1 = (int)((d.y >> 16) / TILE);
            if (shapes) {
                const CullShape cs = cull_shape(rec);
                if (cs.mode == 0) {
                    flags = kRectFull;
                } else if (cs.mode == 2) {
                    keep = false;
                } else {
                    int r1;
                    slab_rows<TILE>(cs, ty0, ty1, r0, r1);
                    nrows = max(0, r1 - r0 + 1);
                    keep = nrows > 0;
                    s_cs[tid] = cs;
                }
            }
        }
    }
    if (shapes) {  // uniform
        s_cmin[tid] = tx1 + 1;
        s_cmax[tid] = tx0 - 1;
        int incl = nrows;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        const int total = __shfl(incl, 63), excl = incl - nrows;
        const bool table = nrows <= kSpanRows;
        int carry = 0;  // the lane whose rows hold the round's first
        for (int base = 0; base < total; base += 64) {
            s_slot[w][lane] = -1;
            __builtin_amdgcn_wave_barrier();
            if (nrows > 0 && excl >= base && excl < base + 64) s_slot[w][excl - base] = lane;
            __builtin_amdgcn_wave_barrier();
            int o = s_slot[w][lane];
            if (lane == 0 && o < 0) o = carry;
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(o, off);
                if (lane >= off) o = max(o, y);
            }
            carry = __shfl(o, 63);
            const int g = max(o, 0);
            const int ex = __shfl(excl, g), gr0 = __shfl(r0, g), gx0 = __shfl(tx0, g), gx1 = __shfl(tx1, g);
            const int gtab = __shfl((int)table, g);
            const int k = base + lane;
            if (k < total) {
                const int gt = (w << 6) + g;
                const uint32_t e = row_span<TILE>(s_cs[gt], gr0 + (k - ex), gx0, gx1);
                if (gtab) spans[((size_t)blockIdx.x * 256 + gt) * kSpanRows + (k - ex)] = e;
                if (e != 0u) {
                    atomicMin(&s_cmin[gt], (int)(e & 0xFFFFu));
                    atomicMax(&s_cmax[gt], (int)(e >> 16) - 1);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (keep && nrows > 0) {
            const int cmin = s_cmin[tid], cmax = s_cmax[tid];
            keep = cmin <= cmax;
            if (keep) {
                tx0 = cmin; tx1 = cmax; ty0 = r0; ty1 = r0 + nrows - 1;
                if (!table) {
                    flags = kRectShape;
                    shapes[j] = s_cs[tid];
                }
            }
        }
    }
    uint32_t c = 0u;
    if (j < n) {
        uint64_t rect = 0ull;
        if (keep) {
            rect = pack_rect((uint32_t)tx0, (uint32_t)tx1, (uint32_t)ty0, (uint32_t)ty1) | flags;
            c = ((uint32_t)tx1 / S - (uint32_t)tx0 / S + 1u) * ((uint32_t)ty1 / S - (uint32_t)ty0 / S + 1u);
        }
        rect_sorted[j] = rect;
        cnt[j] = c;
    }
    unsigned long long tot;
    block_exclusive_scan_256<unsigned long long>((unsigned long long)c, s_buf, tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Counting variant only: (view, Gaussian) pairs of the views [v0, v0 + nv)
// whose pixel square meets the image (the on-screen pairs; a 3D Gaussian's
// record is its view's static_view's), added to *counter.  grid.y: the view.
__global__ void __launch_bounds__(256) k_count_onscreen(const Rec* __restrict__ recs, int N, int n4,
                                                        const ViewParams* __restrict__ views, int v0,
                                                        unsigned long long* counter) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    const int v = v0 + (int)blockIdx.y;
    const int rv = i < n4 ? v : views[v].static_view;
    const bool on = i < N && recs[(size_t)rv * N + i].d.w != 0u;
    const unsigned long long c = (unsigned long long)__popcll(__ballot(on));
    if (__lane_id() == 0 && c) atomicAdd(counter, c);
}

void launch_count_onscreen(const Rec* recs, int N, int n4, const ViewParams* views, int v0, int nv,
                           unsigned long long* counter, hipStream_t st) {
    if (N == 0 || nv == 0) return;
    k_count_onscreen<<<dim3((unsigned)((N + 255) / 256), nv), 256, 0, st>>>(recs, N, n4, views, v0, counter);
}

// offsets[j] = partials[j / 256] (scanned) + this workgroup's exclusive scan;
// run_start as in k_scan_down.
__global__ void __launch_bounds__(256) k_coarse_down(const uint32_t* __restrict__ cnt, int n,
                                                     const unsigned long long* __restrict__ partials, int nparts,
                                                     unsigned long long* __restrict__ offsets,
                                                     uint32_t* __restrict__ run_start, uint64_t run_cap) {
    __shared__ unsigned long long s_buf[256];
    const int j = blockIdx.x * 256 + (int)threadIdx.x;
    const uint32_t c = j < n ? cnt[j] : 0u;
    unsigned long long tot;
    const unsigned long long run =
        block_exclusive_scan_256<unsigned long long>((unsigned long long)c, s_buf, tot) + partials[blockIdx.x];
    if (j < n) {
        offsets[j] = run;
        for (uint64_t r = (run + 255) / 256; r * 256 < run + c && r < run_cap; ++r) run_start[r] = (uint32_t)j;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[n] = partials[nparts];
}

// The capacity check of a pass whose coarse entries total C (one thread): its
// entries take [cbase[v0], cbase[v0] + C) of the call's ccap; the need is
// counted in (Gaussian, tile) slots, S^2 per coarse entry.
__device__ inline void coarse_finalize(unsigned long long C, uint64_t ccap, int S, unsigned long long* cbase, int v0,
                                       int v1, Status* status, unsigned long long* eff_count) {
    const unsigned long long base = cbase[v0];
    status->pairs_needed += C * (unsigned long long)(S * S);
    if (base + C > ccap) {
        status->flags |= kFlagOverflow;
        *eff_count = 0ull;
        cbase[v1] = base;
    } else {
        *eff_count = C;
        cbase[v1] = base + C;
    }
}

// Few count workgroups (nparts <= kDirectParts): k_coarse_top and k_coarse_down
// in one launch.  Each workgroup sums the partials of the workgroups before it
// (workgroup 0 sums them all, finalizes the pass and writes offsets[n]), then
// scans its own counts as k_coarse_down does.
constexpr int kDirectParts = 2048;
__global__ void __launch_bounds__(256) k_coarse_down_direct(const uint32_t* __restrict__ cnt, int n,
                                                            const unsigned long long* __restrict__ partials,
                                                            int nparts, uint64_t ccap, int S,
                                                            unsigned long long* cbase, int v0, int v1,
                                                            Status* status, unsigned long long* eff_count,
                                                            unsigned long long* __restrict__ offsets,
                                                            uint32_t* __restrict__ run_start, uint64_t run_cap) {
    __shared__ unsigned long long s_buf[256];
    const int b = (int)blockIdx.x;
    const int upto = b == 0 ? nparts : b;
    unsigned long long acc = 0;
    for (int i = (int)threadIdx.x; i < upto; i += 256) acc += partials[i];
    unsigned long long sum;
    block_exclusive_scan_256<unsigned long long>(acc, s_buf, sum);
    const unsigned long long before = b == 0 ? 0ull : sum;
    if (b == 0 && threadIdx.x == 0) {
        coarse_finalize(sum, ccap, S, cbase, v0, v1, status, eff_count);
        offsets[n] = sum;
    }
    const int j = b * 256 + (int)threadIdx.x;
    const uint32_t c = j < n ? cnt[j] : 0u;
    unsigned long long tot;
    const unsigned long long run = block_exclusive_scan_256<unsigned long long>((unsigned long long)c, s_buf, tot) + before;
    if (j < n) {
        offsets[j] = run;
        for (uint64_t r = (run + 255) / 256; r * 256 < run + c && r < run_cap; ++r) run_start[r] = (uint32_t)j;
    }
}

// Exclusive scan of the count workgroups' sums (partials[nparts] = total C),
// then the coarse capacity check of the pass (coarse_finalize).
// (1024 threads, each scanning a contiguous chunk of the partials four loads
// at a time: with many count workgroups, e.g. 32 views of 1M Gaussians, this
// single workgroup's walk over the partials is the launch)
__global__ void __launch_bounds__(1024) k_coarse_top(unsigned long long* __restrict__ partials, int nparts,
                                                     uint64_t ccap, int S, unsigned long long* cbase, int v0,
                                                     int v1, Status* status, unsigned long long* eff_count) {
    __shared__ unsigned long long s_w[16];
    const int tid = (int)threadIdx.x, lane = tid & 63, w = tid >> 6;
    // thread t scans the contiguous chunk [t q, (t + 1) q) of the partials
    const int q = (nparts + 1023) / 1024;
    const int i0 = min(nparts, tid * q), i1 = min(nparts, i0 + q);
    unsigned long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int i = i0;
    for (; i + 3 < i1; i += 4) {
        a0 += partials[i];
        a1 += partials[i + 1];
        a2 += partials[i + 2];
        a3 += partials[i + 3];
    }
    for (; i < i1; ++i) a0 += partials[i];
    const unsigned long long sum = (a0 + a1) + (a2 + a3);
    // exclusive scan of the chunk sums over the workgroup (wave scans, then the
    // 16 wave totals)
    unsigned long long incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    unsigned long long run = incl - sum, carry = 0;
    for (int k = 0; k < 16; ++k) {
        const unsigned long long t = s_w[k];
        if (k < w) run += t;
        carry += t;
    }
    for (i = i0; i + 3 < i1; i += 4) {
        const unsigned long long v0_ = partials[i], v1_ = partials[i + 1], v2_ = partials[i + 2], v3_ = partials[i + 3];
        partials[i] = run;
        partials[i + 1] = run + v0_;
        partials[i + 2] = run + v0_ + v1_;
        partials[i + 3] = run + v0_ + v1_ + v2_;
        run += v0_ + v1_ + v2_ + v3_;
    }
    for (; i < i1; ++i) {
        const unsigned long long v = partials[i];
        partials[i] = run;
        run += v;
    }
    if (tid != 0) return;
    partials[nparts] = carry;
    coarse_finalize(carry, ccap, S, cbase, v0, v1, status, eff_count);
}

// Coarse entries (super-tile id relative to the pass's first, depth rank j),
// written in (segment, depth) order: one thread per entry, which finds its
// Gaussian by binary search over the count offsets (entries, not Gaussians,
// are spread evenly: the nearest splats are the largest and sit together in
// depth order).  The key's upper 16 bits carry the entry's tile mask (the
// super-tile sort reads only the low bits); shapes != null applies the alpha
// >= 1/255 tile test.
template <int TILE>
__global__ void __launch_bounds__(256) k_coarse_emit(const unsigned long long* __restrict__ offsets,
                                                     const uint32_t* __restrict__ run_start, int n, SegLayout sg,
                                                     const uint64_t* __restrict__ rect_sorted,
                                                     const CullShape* __restrict__ shapes,
                                                     const uint32_t* __restrict__ spans,
                                                     const ViewParams* __restrict__ views, int v0,
                                                     const unsigned long long* eff_count,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    constexpr uint32_t S = (uint32_t)super_factor(TILE);
    __shared__ unsigned long long s_off[257];
    const uint64_t C = *eff_count;
    const int tid = threadIdx.x;
    // blocks take runs of 256 consecutive entries (run_start names the Gaussian
    // holding a run's first entry); within a segment invisible
    // Gaussians sort last (culled key), so the visible ones all own entries and
    // a run usually spans at most 256 consecutive Gaussians (entries past the
    // block's window, after another segment's invisible tail, search globally)
    for (uint64_t p0 = (uint64_t)blockIdx.x * 256; p0 < C; p0 += (uint64_t)gridDim.x * 256) {
        const int j0 = (int)run_start[p0 / 256];  // Gaussian holding entry p0
        s_off[tid] = offsets[min(j0 + tid, n)];
        if (tid == 0) s_off[256] = offsets[min(j0 + 256, n)];
        __syncthreads();
        const uint64_t p = p0 + tid;
        if (p < C) {
            int j;
            unsigned long long pj;  // offsets[j]
            if (p < s_off[256]) {
                int lo = 0, hi = 256;  // last k with s_off[k] <= p
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= p) lo = mid; else hi = mid;
                }
                j = j0 + lo;
                pj = s_off[lo];
            } else {
                int lo = min(j0 + 256, n - 1), hi = n;  // offsets[lo] <= p < offsets[n]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (offsets[mid] <= p) lo = mid; else hi = mid;
                }
                j = lo;
                pj = offsets[lo];
            }
            const SegPos sp = seg_of(j, sg, views, v0);
            const ViewParams& V = views[sp.view];
            const uint64_t rf = rect_sorted[j], r = rf & kRectCoords;
            const uint32_t tx0 = (uint32_t)(r & 0xFFFFu), tx1 = (uint32_t)((r >> 16) & 0xFFFFu);
            const uint32_t ty0 = (uint32_t)((r >> 32) & 0xFFFFu), ty1 = (uint32_t)(r >> 48);
            const uint32_t sx0 = tx0 / S, sw = tx1 / S - sx0 + 1u, sy0 = ty0 / S;
            // (row, column) of the entry in the splat's sw-wide block of
            // super-tiles: a float quotient, exact after one correction
            // (local < 2^24)
            const uint32_t local = (uint32_t)(p - pj);
            uint32_t sy = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)sw));
            if (sy * sw > local) --sy;
            else if ((sy + 1u) * sw <= local) ++sy;
            const uint32_t sx = local - sy * sw;
            uint32_t key = (uint32_t)sp.super0 + (sy0 + sy) * (uint32_t)V.sx + sx0 + sx;
            const uint32_t bx = (sx0 + sx) * S, by = (sy0 + sy) * S;
            uint32_t m;
            if (!shapes || (rf & kRectFull)) {
                m = tile_mask<TILE>(CullShape{}, false, tx0, tx1, ty0, ty1, bx, by);
            } else if (rf & kRectShape) {
                m = tile_mask<TILE>(shapes[j], true, tx0, tx1, ty0, ty1, bx, by);
            } else {
                m = span_mask<TILE>(spans + (size_t)j * kSpanRows, ty0, ty1, bx, by);
            }
            key |= m << 16;
            keys[p] = key;
            vals[p] = (uint32_t)j;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ keys, uint32_t key_mask,
                                                const unsigned long long* eff_count,
                                                const unsigned long long* base_ptr, int64_t* __restrict__ ranges) {
    const uint64_t n = *eff_count;
    const int64_t base = base_ptr ? (int64_t)*base_ptr : 0;
    keys += base;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = keys[i] & key_mask;
        if (i == 0 || (keys[i - 1] & key_mask) != t) ranges[2 * (size_t)t] = base + (int64_t)i;
        if (i + 1 == n || (keys[i + 1] & key_mask) != t) ranges[2 * (size_t)t + 1] = base + (int64_t)i + 1;
    }
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = val;
}
// Backward: workgroup k < passes.n (order_blocks = passes.n) orders pass k
// from the forward's per-bucket tile counts (an exclusive scan, then one
// scatter pass over the tiles; ties in any order), or, with order_blocks = 0,
// the order comes from a sort (k_bwd_order_keys); the other workgroups zero g2
// when a backward has used it since the forward (*dirty) or when force is set.
// Counts that do not add up to the pass's tiles give the identity order.
__global__ void __launch_bounds__(1024) k_bwd_prologue(float* __restrict__ g2, size_t n_g2,
                                                       const unsigned long long* __restrict__ dirty, int force,
                                                       const uint32_t* __restrict__ tcost,
                                                       const uint32_t* __restrict__ thist, PassTiles passes,
                                                       int order_blocks, uint32_t* __restrict__ order) {
    const int k = (int)blockIdx.x;
    if (k < order_blocks) {
        __shared__ uint32_t s_pos[kCostBuckets];
        __shared__ uint32_t s_total, s_bad;
        static_assert(kCostBuckets == 16 * 64, "one wave scans the buckets");
        const int tid = threadIdx.x, nt = blockDim.x;
        const int t0 = passes.tile0[k], n = passes.tile0[k + 1] - t0;
        const uint32_t* h = thist + (size_t)k * kCostBuckets;
        order += t0;
        if (tid < 64) {
            uint32_t v[16], sum = 0u;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                v[i] = h[16 * tid + i];
                sum += v[i];
            }
            uint32_t incl = sum;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = (uint32_t)__shfl_up((int)incl, off);
                if (tid >= off) incl += y;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                s_pos[16 * tid + i] = run;
                run += v[i];
            }
            if (tid == 63) s_total = run;
        }
        if (tid == 0) s_bad = 0u;
        __syncthreads();
        if (s_total == (uint32_t)n) {
            for (int t = tid; t < n; t += nt) {
                const uint32_t pos = atomicAdd(&s_pos[cost_bucket(tcost[t0 + t])], 1u);
                if (pos < (uint32_t)n) order[pos] = (uint32_t)t;
                else s_bad = 1u;
            }
        }
        __syncthreads();
        if (s_total != (uint32_t)n || s_bad)
            for (int t = tid; t < n; t += nt) order[t] = (uint32_t)t;
        return;
    }
    if (!force && *dirty == 0ull) return;  // the records are as the forward left them (uniform)
    const size_t nb = (size_t)(gridDim.x - order_blocks);
    const size_t i0 = (size_t)(k - order_blocks) * blockDim.x + threadIdx.x, step = nb * blockDim.x;
    if ((reinterpret_cast<uintptr_t>(g2) & 15u) == 0 && (n_g2 & 3) == 0) {  // 16-byte stores
        float4* g4 = reinterpret_cast<float4*>(g2);
        for (size_t i = i0; i < n_g2 / 4; i += step) g4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    } else {
        for (size_t i = i0; i < n_g2; i += step) g2[i] = 0.0f;
    }
}

// Sort keys of the backward's tile order when a pass has too many tiles for one
// workgroup: per global tile t of pass k, key (k, cost bucket), value t - tile0[k].
__global__ void __launch_bounds__(256) k_bwd_order_keys(const uint32_t* __restrict__ tcost, PassTiles passes,
                                                        uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int t = blockIdx.x * 256 + (int)threadIdx.x;
    if (t >= passes.tile0[passes.n]) return;
    int k = 0;
    while (k + 1 < passes.n && passes.tile0[k + 1] <= t) ++k;
    keys[t] = ((uint32_t)k << 10) | cost_bucket(tcost[t]);
    vals[t] = (uint32_t)(t - passes.tile0[k]);
}

__global__ void k_fill_f32(float* p, size_t n, float val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = val;
}

int coarse_count_blocks(int n) { return ceil_div(n, 256); }
void launch_coarse_count(const uint32_t* sorted_gid, int n, int N, SegLayout sg, const Rec* recs,
                         const ViewParams* views, int v0, int tile, int S, uint32_t* cnt, uint64_t* rect_sorted,
                         CullShape* shapes, uint32_t* spans, unsigned long long* partials, hipStream_t st) {
    if (n == 0) return;
    const int nb = coarse_count_blocks(n);
#define H4D_COARSE_COUNT(T) \
    k_coarse_count<T><<<nb, 256, 0, st>>>(sorted_gid, n, N, sg, recs, views, v0, cnt, rect_sorted, shapes, spans, partials)
    if (tile == 8) H4D_COARSE_COUNT(8);
    else if (tile == 16) H4D_COARSE_COUNT(16);
    else H4D_COARSE_COUNT(32);
#undef H4D_COARSE_COUNT
}
void launch_coarse_offsets(const uint32_t* cnt, int n, unsigned long long* partials, uint64_t ccap, int S,
                           unsigned long long* cbase, int v0, int v1, Status* status, unsigned long long* eff_count,
                           unsigned long long* offsets, uint32_t* run_start, uint64_t run_cap, hipStream_t st) {
    const int nb = coarse_count_blocks(n);
    if (n > 0 && nb <= kDirectParts) {
        k_coarse_down_direct<<<nb, 256, 0, st>>>(cnt, n, partials, nb, ccap, S, cbase, v0, v1, status, eff_count,
                                                 offsets, run_start, run_cap);
        return;
    }
    k_coarse_top<<<1, 1024, 0, st>>>(partials, nb, ccap, S, cbase, v0, v1, status, eff_count);
    if (n > 0) k_coarse_down<<<nb, 256, 0, st>>>(cnt, n, partials, nb, offsets, run_start, run_cap);
}
void launch_coarse_emit(const unsigned long long* offsets, const uint32_t* run_start, int n, SegLayout sg,
                        const uint64_t* rect_sorted, const CullShape* shapes, const uint32_t* spans,
                        const ViewParams* views, int v0, int tile, int S, uint64_t capacity,
                        const unsigned long long* eff_count, uint32_t* keys, uint32_t* vals, hipStream_t st) {
    if (n == 0 || capacity == 0) return;
    // (32 views of 1M Gaussians in one pass: about 25 runs of 256 entries per workgroup)
    const int nb = (int)std::min<uint64_t>(65536, (capacity + 255) / 256);
#define H4D_COARSE_EMIT(T) \
    k_coarse_emit<T><<<nb, 256, 0, st>>>(offsets, run_start, n, sg, rect_sorted, shapes, spans, views, v0, eff_count, \
                                         keys, vals)
    if (tile == 8) H4D_COARSE_EMIT(8);
    else if (tile == 16) H4D_COARSE_EMIT(16);
    else H4D_COARSE_EMIT(32);
#undef H4D_COARSE_EMIT
}
void launch_ranges(const uint32_t* keys, uint32_t key_mask, const unsigned long long* eff_count,
                   const unsigned long long* base, int64_t* ranges, hipStream_t st) {
    k_ranges<<<2048, 256, 0, st>>>(keys, key_mask, eff_count, base, ranges);
}
bool launch_bwd_prologue(float* g2, size_t n_g2, const unsigned long long* dirty, int force, const uint32_t* tcost,
                         const uint32_t* thist, const PassTiles& passes, const OrderSort& sort, uint32_t* order,
                         hipStream_t st) {
    int most = 0;
    for (int k = 0; k < passes.n; ++k) most = std::max(most, passes.tile0[k + 1] - passes.tile0[k]);
    const bool by_sort = most > kOrderBlockTiles;
    // a grid-stride loop of 16-byte stores over at most 4096 workgroups (which
    // return at once when nothing is to be cleared)
    const int fill = (int)std::max<size_t>(1, std::min<size_t>(4096, (n_g2 + 4095) / 4096));
    const int ob = by_sort ? 0 : passes.n;
    k_bwd_prologue<<<ob + fill, 1024, 0, st>>>(g2, n_g2, dirty, force, tcost, thist, passes, ob, order);
    if (!by_sort) return true;
    // one stable sort of (pass, cost bucket) keys over all tiles: every pass's
    // tiles in a run of their own, by decreasing cost
    const int tiles = passes.tile0[passes.n];
    k_bwd_order_keys<<<(tiles + 255) / 256, 256, 0, st>>>(tcost, passes, sort.keys, sort.vals);
    int bits = 10;
    while ((1 << (bits - 10)) < passes.n) ++bits;
    const int np = (bits + kMaxRadixBits - 1) / kMaxRadixBits;
    uint32_t *kin = sort.keys, *vin = sort.vals, *kalt = sort.keys2, *valt = sort.vals2;
    for (int p = 0, shift = 0; p < np; ++p) {
        const int nb = (bits - shift + (np - p) - 1) / (np - p);
        uint32_t* vout = p == np - 1 ? order : valt;
        if (!launch_radix_pass(kin, vin, kalt, vout, nullptr, (uint64_t)tiles, (uint64_t)tiles, shift, nb, sort.hist,
                               sort.hist_words, sort.totals, sort.totals_words, nullptr, st))
            return false;
        std::swap(kin, kalt);
        vin = vout;
        valt = (vout == sort.vals2) ? sort.vals : sort.vals2;
        shift += nb;
    }
    return true;
}

void launch_fill_u64(unsigned long long* p, size_t n, unsigned long long val, hipStream_t st) {
    if (n == 0) return;
    const int nb = (int)std::min<size_t>(4096, (n + 255) / 256);
    k_fill_u64<<<nb, 256, 0, st>>>(p, n, val);
}
void launch_fill_f32(float* p, size_t n, float val, hipStream_t st) {
    if (n == 0) return;
    const int nb = (int)std::min<size_t>(8192, (n + 255) / 256);
    k_fill_f32<<<nb, 256, 0, st>>>(p, n, val);
}

}  // namespace h4d

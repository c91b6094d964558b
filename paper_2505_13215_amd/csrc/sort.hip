// Binning and ordering on gfx950 (Alg. 1: DuplicateWithKeys, SortByKeys,
// IdentifyTileRanges).
//
// Design: the per-view depth order is established once over the N Gaussians
// (LSD radix sort of the float32 depth bits, stable, so equal depths keep
// ascending id), pairs are then emitted in that order and only the tile id is
// sorted (a stable LSD radix sort over ceil(log2(tiles)) bits).  Stability makes
// the final order exactly (tile, depth bits, id) while moving 8 bytes per pair
// per pass instead of sorting 64-bit (tile, depth) keys.
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
    const int tid = threadIdx.x;
    s_buf[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        T add = tid >= off ? s_buf[tid - off] : (T)0;
        __syncthreads();
        s_buf[tid] += add;
        __syncthreads();
    }
    total = s_buf[255];
    const T incl = s_buf[tid];
    __syncthreads();
    return incl - v;
}

// ---------------------------------------------------------------------------
// Radix sort pass
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSortThreads) k_radix_upsweep(const uint32_t* __restrict__ keys,
                                                                const unsigned long long* dcount, uint64_t hcount,
                                                                int shift, int nbits, uint32_t* __restrict__ hist,
                                                                int nblocks) {
    __shared__ uint32_t s_hist[4][256];
    const int radix = 1 << nbits;
    const uint32_t mask = (uint32_t)radix - 1u;
    const int tid = threadIdx.x, w = tid >> 6;
    for (int d = tid; d < 4 * 256; d += kSortThreads) (&s_hist[0][0])[d] = 0;
    __syncthreads();
    const uint64_t n = read_count(dcount, hcount);
    const uint64_t begin = (uint64_t)blockIdx.x * kSortTile;
    if (begin < n) {
        for (int k = 0; k < kSortItems; ++k) {
            const uint64_t idx = begin + (uint64_t)k * kSortThreads + tid;
            if (idx < n) atomicAdd(&s_hist[w][(keys[idx] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < radix; d += kSortThreads)
        hist[(size_t)d * nblocks + blockIdx.x] = s_hist[0][d] + s_hist[1][d] + s_hist[2][d] + s_hist[3][d];
}

// one block per digit: exclusive scan of that digit's per-block counts
__global__ void __launch_bounds__(256) k_radix_digit_scan(uint32_t* __restrict__ hist, int nblocks,
                                                          uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_buf[256];
    uint32_t* h = hist + (size_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    for (int start = 0; start < nblocks; start += 256) {
        const int i = start + threadIdx.x;
        const uint32_t v = i < nblocks ? h[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan_256<uint32_t>(v, s_buf, tot);
        if (i < nblocks) h[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kSortThreads) k_radix_downsweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const unsigned long long* dcount, uint64_t hcount, int shift, int nbits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int nblocks,
    const unsigned long long* out_offset) {
    __shared__ uint32_t s_wcount[4][256];
    __shared__ uint32_t s_dstart[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_scan[256];
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];

    const uint64_t n = read_count(dcount, hcount);
    const uint64_t begin = (uint64_t)blockIdx.x * kSortTile;
    if (begin >= n) return;  // uniform over the block
    const int radix = 1 << nbits;
    const uint32_t mask = (uint32_t)radix - 1u;
    const int tid = threadIdx.x, w = tid >> 6, lane = __lane_id();

    for (int d = tid; d < 4 * 256; d += kSortThreads) (&s_wcount[0][0])[d] = 0;
    // global base of digit d = (exclusive scan of totals)[d] + this block's scanned count
    uint32_t tot;
    const uint32_t tv = tid < radix ? totals[tid] : 0u;
    const uint32_t dbase = block_exclusive_scan_256<uint32_t>(tv, s_scan, tot);
    if (tid < radix) s_gbase[tid] = dbase + hist[(size_t)tid * nblocks + blockIdx.x];
    __syncthreads();

    // wave w owns items [begin + w*512, begin + (w+1)*512), 8 rounds of 64
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
    const unsigned long long lt = lanemask_lt();
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t idx = begin + (uint64_t)w * (kSortItems * 64) + (uint64_t)r * 64 + lane;
        const bool valid = idx < n;
        key[r] = valid ? keys_in[idx] : 0u;
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
    // per digit: prefix over waves; block total per digit
    uint32_t dt = 0;
    if (tid < radix) {
        uint32_t run = 0;
        for (int q = 0; q < 4; ++q) {
            const uint32_t c = s_wcount[q][tid];
            s_wcount[q][tid] = run;
            run += c;
        }
        dt = run;
    }
    uint32_t blk_tot;
    const uint32_t ds = block_exclusive_scan_256<uint32_t>(dt, s_scan, blk_tot);
    if (tid < radix) s_dstart[tid] = ds;
    __syncthreads();
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t idx = begin + (uint64_t)w * (kSortItems * 64) + (uint64_t)r * 64 + lane;
        if (idx < n) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t pos = s_dstart[d] + s_wcount[w][d] + rank[r];
            s_keys[pos] = key[r];
            s_vals[pos] = val[r];
        }
    }
    __syncthreads();
    const int cnt = (int)min((uint64_t)kSortTile, n - begin);
    const unsigned long long off = out_offset ? *out_offset : 0ull;
    for (int p = tid; p < cnt; p += kSortThreads) {
        const uint32_t k = s_keys[p];
        const uint32_t d = (k >> shift) & mask;
        const uint64_t dst = (uint64_t)s_gbase[d] + (uint64_t)(p - (int)s_dstart[d]);
        keys_out[dst] = k;
        vals_out[dst + off] = s_vals[p];
    }
}

int radix_blocks(uint64_t capacity) { return (int)((capacity + kSortTile - 1) / kSortTile); }
size_t radix_hist_words(uint64_t capacity) { return (size_t)256 * (size_t)std::max(1, radix_blocks(capacity)); }

void launch_radix_pass(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
                       const unsigned long long* dcount, uint64_t hcount, uint64_t capacity, int shift, int nbits,
                       uint32_t* hist, uint32_t* totals, const unsigned long long* out_offset, hipStream_t st) {
    const int nb = radix_blocks(capacity);
    if (nb == 0) return;
    k_radix_upsweep<<<nb, kSortThreads, 0, st>>>(keys_in, dcount, hcount, shift, nbits, hist, nb);
    k_radix_digit_scan<<<1 << nbits, 256, 0, st>>>(hist, nb, totals);
    k_radix_downsweep<<<nb, kSortThreads, 0, st>>>(keys_in, vals_in, keys_out, vals_out, dcount, hcount, shift, nbits,
                                                    hist, totals, nb, out_offset);
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

__global__ void __launch_bounds__(256) k_scan_down(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx,
                                                   int n, const unsigned long long* __restrict__ partials, int nparts,
                                                   unsigned long long* __restrict__ out) {
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
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partials[nparts];
}

int scan_blocks(int n) { return (n + kScanTile - 1) / kScanTile; }

void launch_scan_u32_u64(const uint32_t* in, const uint32_t* idx, int n, unsigned long long* out,
                         unsigned long long* partials, hipStream_t st) {
    const int nb = std::max(1, scan_blocks(n));
    k_scan_reduce<<<nb, 256, 0, st>>>(in, idx, n, partials);
    k_scan_top<<<1, 256, 0, st>>>(partials, nb);
    k_scan_down<<<nb, 256, 0, st>>>(in, idx, n, partials, nb, out);
}

// ---------------------------------------------------------------------------
// Pair bookkeeping, emission, ranges.
// ---------------------------------------------------------------------------
__global__ void k_finalize_pairs(const unsigned long long* offsets, int n, unsigned long long* pair_base, int view,
                                 uint64_t capacity, Status* status, unsigned long long* eff_count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long P = offsets[n];
    const unsigned long long base = pair_base[view];
    status->pairs_needed += P;
    if (base + P > capacity) {
        status->flags |= kFlagOverflow;
        *eff_count = 0ull;
        pair_base[view + 1] = base;
    } else {
        *eff_count = P;
        pair_base[view + 1] = base + P;
    }
}

// One block per 256 depth-ordered Gaussians; threads stride over the block's
// contiguous pair range and find their Gaussian by binary search in LDS, so the
// key/value writes are coalesced.
__global__ void __launch_bounds__(256) k_emit(const uint32_t* __restrict__ sorted_gid,
                                              const unsigned long long* __restrict__ offsets, int n,
                                              const Rec* __restrict__ recs, int tile, int tiles_x,
                                              const unsigned long long* eff_count, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals) {
    __shared__ unsigned long long s_off[257];
    __shared__ uint32_t s_gid[256], s_tx0[256], s_ty0[256], s_tw[256];
    if (*eff_count == 0ull) return;
    const int tid = threadIdx.x;
    const int j0 = blockIdx.x * 256;
    const int j = j0 + tid;
    if (j < n) {
        const uint32_t g = sorted_gid[j];
        s_gid[tid] = g;
        s_off[tid] = offsets[j];
        const uint4 d = recs[g].d;
        const uint32_t x0 = d.x & 0xFFFFu, x1 = d.x >> 16, y0 = d.y & 0xFFFFu;
        s_tx0[tid] = x0 / (uint32_t)tile;
        s_tw[tid] = x1 / (uint32_t)tile - x0 / (uint32_t)tile + 1u;
        s_ty0[tid] = y0 / (uint32_t)tile;
    } else {
        s_off[tid] = offsets[n];
        s_gid[tid] = 0; s_tx0[tid] = 0; s_tw[tid] = 1; s_ty0[tid] = 0;
    }
    if (tid == 0) s_off[256] = offsets[min(j0 + 256, n)];
    __syncthreads();
    const unsigned long long start = s_off[0], end = s_off[256];
    for (unsigned long long p = start + tid; p < end; p += 256) {
        // last k with s_off[k] <= p
        int lo = 0, hi = 256;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= p) lo = mid; else hi = mid;
        }
        const uint32_t local = (uint32_t)(p - s_off[lo]);
        const uint32_t tw = s_tw[lo];
        const uint32_t ty = local / tw, tx = local - ty * tw;
        keys[p] = (s_ty0[lo] + ty) * (uint32_t)tiles_x + s_tx0[lo] + tx;
        vals[p] = s_gid[lo];
    }
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ keys, const unsigned long long* eff_count,
                                                const unsigned long long* base_ptr, int64_t* __restrict__ ranges) {
    const uint64_t n = *eff_count;
    const int64_t base = (int64_t)*base_ptr;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t t = keys[i];
        if (i == 0 || keys[i - 1] != t) ranges[2 * (size_t)t] = base + (int64_t)i;
        if (i + 1 == n || keys[i + 1] != t) ranges[2 * (size_t)t + 1] = base + (int64_t)i + 1;
    }
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = val;
}
__global__ void k_fill_f32(float* p, size_t n, float val) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = val;
}
__global__ void k_zero_status(Status* s, unsigned long long* pair_base, int n_views) {
    const int t = threadIdx.x;
    if (t < 8) (&s->flags)[t] = 0ull;
    for (int v = t; v <= n_views; v += blockDim.x) pair_base[v] = 0ull;
}

void launch_finalize_pairs(const unsigned long long* offsets, int n, unsigned long long* pair_base, int view,
                           uint64_t capacity, Status* status, unsigned long long* eff_count, hipStream_t st) {
    k_finalize_pairs<<<1, 1, 0, st>>>(offsets, n, pair_base, view, capacity, status, eff_count);
}
void launch_emit(const uint32_t* sorted_gid, const unsigned long long* offsets, int n, const Rec* recs, int tile,
                 int tiles_x, const unsigned long long* eff_count, uint32_t* keys, uint32_t* vals, hipStream_t st) {
    if (n == 0) return;
    k_emit<<<ceil_div(n, 256), 256, 0, st>>>(sorted_gid, offsets, n, recs, tile, tiles_x, eff_count, keys, vals);
}
void launch_ranges(const uint32_t* keys, const unsigned long long* eff_count, const unsigned long long* base,
                   int64_t* ranges, hipStream_t st) {
    k_ranges<<<2048, 256, 0, st>>>(keys, eff_count, base, ranges);
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
void launch_zero_status(Status* s, unsigned long long* pair_base, int n_views, hipStream_t st) {
    k_zero_status<<<1, 64, 0, st>>>(s, pair_base, n_views);
}

}  // namespace h4d

// Front-to-back blending on gfx950 (Eq. 3; Alg. 1 BlendInOrder) and its adjoint.
//
// One workgroup per B x B tile (B = 8 and 16: one wave64; 32: four waves), one or
// four pixels per lane.  The tile's depth-ordered list is walked in chunks: each
// chunk of records is gathered once from HBM into LDS and broadcast to every lane.
// A pixel's contributors are exactly the splats whose pixel square contains it,
// so the image does not depend on B or on the chunk size.
//
// The backward recomputes transmittance front to back with the very same
// blending step as the forward (eval_splat), takes the colour behind a splat as
// C_out minus the running prefix, sums each lane's pixels in registers, reduces
// the nine per-splat gradients across the wave with DPP (skipped when no lane
// blended the splat), parks the wave sums in the register file and flushes them
// with one global atomic per (splat, component, wave).  Each wave stops at its
// own last contributor.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

// LDS copy of one record (64 bytes, 16-byte aligned so that a lane reads it
// with four 128-bit LDS loads): packed pixel square, centre split into integer
// and fractional parts, scaled conic, opacity, colour.
struct __align__(16) LSplat {
    uint32_t rx, ry;              // x0 | x1 << 16, y0 | y1 << 16
    float ui, uf, vi, vf;
    float qa, qb, qc, op;
    float cr, cg, cb;
    uint32_t pad[3];
};
static_assert(sizeof(LSplat) == 64, "LDS splat is 64 bytes");

__device__ __forceinline__ void stage_splat(const Rec& r, LSplat& s) {
    s.rx = r.d.x; s.ry = r.d.y;
    s.ui = r.c.y; s.uf = r.a.x; s.vi = r.c.z; s.vf = r.a.y;
    s.qa = r.a.z; s.qb = r.a.w; s.qc = r.b.x; s.op = r.b.y;
    s.cr = r.b.z; s.cg = r.b.w; s.cb = r.c.x;
}

__device__ __forceinline__ Splat to_splat(const LSplat& l) {
    Splat s;
    s.x0 = (int)(l.rx & 0xFFFFu); s.x1 = (int)(l.rx >> 16); s.y0 = (int)(l.ry & 0xFFFFu); s.y1 = (int)(l.ry >> 16);
    s.ui = l.ui; s.uf = l.uf; s.vi = l.vi; s.vf = l.vf;
    s.qa = l.qa; s.qb = l.qb; s.qc = l.qc; s.op = l.op;
    s.cr = l.cr; s.cg = l.cg; s.cb = l.cb;
    return s;
}

__device__ __forceinline__ bool in_square(const Splat& s, int px, int py) {
    return px >= s.x0 && px <= s.x1 && py >= s.y0 && py <= s.y1;
}

// Lane layout: a 16 x 16 tile is one wave, every lane holding four pixels
// (rows r, r + 4, r + 8, r + 12 of its column); 8 x 8 is one wave with one pixel
// per lane; 32 x 32 is four waves with four pixels per lane.  The per-splat LDS
// reads, loop control and (backward) cross-lane reductions are shared by all of
// a lane's pixels.
template <int B>
struct Shape {
    static constexpr int NT = (B == 32) ? 256 : 64;  // threads per tile
    static constexpr int PPL = B * B / NT;           // pixels per lane
};

// STATS = true is a measurement-only instantiation that also counts (pixel,
// splat) evaluations and blends into counters[0..1].
template <int B, int CHUNK, bool STATS>
__global__ void __launch_bounds__(Shape<B>::NT) k_composite_fwd(
    const Rec* __restrict__ recs, int N, const uint32_t* __restrict__ ids, const int64_t* __restrict__ ranges,
    const ViewParams* __restrict__ views, int v0, int v1, PtrTable images, float* __restrict__ Tfin,
    uint32_t* __restrict__ ncontrib, float* __restrict__ Cout, unsigned long long* counters) {
    constexpr int NT = Shape<B>::NT, PPL = Shape<B>::PPL;
    __shared__ LSplat s_sp[CHUNK];
    const int gt = views[v0].tile_base + (int)blockIdx.x;
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    recs += (size_t)view * N;
    float* __restrict__ image = images.p[view];
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    int px[PPL], py[PPL];
    float pxc[PPL], pyc[PPL], T[PPL], cr[PPL], cg[PPL], cb[PPL];
    uint32_t last[PPL];
    bool done[PPL];
    bool lane_done = true;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = (int)threadIdx.x + k * NT;
        px[k] = tx * B + p % B;
        py[k] = ty * B + p / B;
        pxc[k] = (float)px[k] + 0.5f;
        pyc[k] = (float)py[k] + 0.5f;
        T[k] = 1.0f;
        cr[k] = cg[k] = cb[k] = 0.f;
        last[k] = 0u;
        done[k] = !(px[k] < V.W && py[k] < V.H);
        lane_done = lane_done && done[k];
    }
    const int64_t start = ranges[2 * (size_t)(V.tile_base + tile)];
    const int64_t end = ranges[2 * (size_t)(V.tile_base + tile) + 1];
    unsigned long long n_eval = 0, n_blend = 0;
    for (int64_t base = start; base < end; base += CHUNK) {
        if (__syncthreads_count(lane_done) == NT) break;
        const int cnt = (int)min((int64_t)CHUNK, end - base);
        for (int k = threadIdx.x; k < cnt; k += NT) stage_splat(recs[ids[base + k]], s_sp[k]);
        __syncthreads();
        if (!lane_done) {
            const uint32_t rel0 = (uint32_t)(base - start);
            for (int j = 0; j < cnt; ++j) {
                const Splat s = to_splat(s_sp[j]);
                bool all = true;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    float dx, dy, G, alpha;
                    bool clamped;
                    const bool ok = eval_splat(s, px[k], py[k], pxc[k], pyc[k], dx, dy, G, alpha, clamped) && !done[k];
                    const float Tn = next_T(T[k], alpha);
                    const bool stop = ok && Tn < kMinT;
                    const bool bl = ok && !stop;
                    const float w = bl ? alpha * T[k] : 0.0f;
                    cr[k] = __builtin_fmaf(s.cr, w, cr[k]);
                    cg[k] = __builtin_fmaf(s.cg, w, cg[k]);
                    cb[k] = __builtin_fmaf(s.cb, w, cb[k]);
                    T[k] = bl ? Tn : T[k];
                    last[k] = bl ? rel0 + (uint32_t)j + 1u : last[k];
                    if (STATS) {
                        n_eval += (!done[k] && in_square(s, px[k], py[k])) ? 1u : 0u;
                        n_blend += bl ? 1u : 0u;
                    }
                    done[k] = done[k] || stop;
                    all = all && done[k];
                }
                if (all) {
                    lane_done = true;
                    break;
                }
            }
        }
    }
    const size_t HW = (size_t)V.W * V.H;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (px[k] < V.W && py[k] < V.H) {
            const size_t p = (size_t)py[k] * V.W + px[k];
            const float o0 = __builtin_fmaf(T[k], V.bg[0], cr[k]), o1 = __builtin_fmaf(T[k], V.bg[1], cg[k]),
                        o2 = __builtin_fmaf(T[k], V.bg[2], cb[k]);
            image[p] = o0;
            image[HW + p] = o1;
            image[2 * HW + p] = o2;
            const size_t q = (size_t)V.pix_base + p;
            Tfin[q] = T[k];
            ncontrib[q] = last[k];
            Cout[3 * (size_t)V.pix_base + p] = o0;
            Cout[3 * (size_t)V.pix_base + HW + p] = o1;
            Cout[3 * (size_t)V.pix_base + 2 * HW + p] = o2;
        }
    }
    if (STATS) {
        atomicAdd(&counters[0], n_eval);
        atomicAdd(&counters[1], n_blend);
    }
}

// Sum over the 64 lanes of a wave, complete in lane 63: quad xor1, quad xor2,
// half-row mirror and row mirror give every lane its row's sum, then two row
// broadcasts fold rows 0-2 into row 3.
__device__ __forceinline__ float wave_sum_to_63(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));
    return v;
}

// Largest value over the wave.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off));
    return v;
}

// Per-splat gradient sums of the current group of 64 splats live in the
// register file: the wave sum of splat j is written into lane j % 64 of nine
// accumulator registers; every 64 splats (and at the end of a chunk) all lanes
// flush their sums with parallel global atomics.
template <int B, int CHUNK, bool STATS>
__global__ void __launch_bounds__(Shape<B>::NT) k_composite_bwd(
    const Rec* __restrict__ recs, int N, const uint32_t* __restrict__ ids, const int64_t* __restrict__ ranges,
    const ViewParams* __restrict__ views, int v0, int v1, CPtrTable dls, const float* __restrict__ Tfin,
    const uint32_t* __restrict__ ncontrib, const float* __restrict__ Cout, float* __restrict__ g2,
    unsigned long long* counters) {
    constexpr int NT = Shape<B>::NT, PPL = Shape<B>::PPL;
    __shared__ LSplat s_sp[CHUNK];
    __shared__ uint32_t s_gid[CHUNK];
    __shared__ uint32_t s_max;
    const int gt = views[v0].tile_base + (int)blockIdx.x;
    const int view = find_view_of_tile(views, v0, v1, gt);
    const ViewParams& V = views[view];
    const int tile = gt - V.tile_base;
    recs += (size_t)view * N;
    g2 += (size_t)view * 9 * N;
    const float* __restrict__ dl = dls.p[view];
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    const int64_t start = ranges[2 * (size_t)(V.tile_base + tile)];
    const size_t HW = (size_t)V.W * V.H;
    const int lane = __lane_id();
    int px[PPL], py[PPL];
    float pxc[PPL], pyc[PPL], G0[PPL], G1[PPL], G2[PPL], C0[PPL], C1[PPL], C2[PPL];
    float T[PPL], pr[PPL], pg[PPL], pb[PPL];
    uint32_t nc[PPL];
    uint32_t lane_nc = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int p = (int)threadIdx.x + k * NT;
        px[k] = tx * B + p % B;
        py[k] = ty * B + p / B;
        pxc[k] = (float)px[k] + 0.5f;
        pyc[k] = (float)py[k] + 0.5f;
        G0[k] = G1[k] = G2[k] = C0[k] = C1[k] = C2[k] = 0.f;
        nc[k] = 0u;
        if (px[k] < V.W && py[k] < V.H) {
            const size_t q = (size_t)py[k] * V.W + px[k];
            G0[k] = dl[q]; G1[k] = dl[HW + q]; G2[k] = dl[2 * HW + q];
            C0[k] = Cout[3 * (size_t)V.pix_base + q];
            C1[k] = Cout[3 * (size_t)V.pix_base + HW + q];
            C2[k] = Cout[3 * (size_t)V.pix_base + 2 * HW + q];
            nc[k] = ncontrib[(size_t)V.pix_base + q];
        }
        T[k] = 1.0f;
        pr[k] = pg[k] = pb[k] = 0.f;
        lane_nc = max(lane_nc, nc[k]);
    }
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    if (lane_nc) atomicMax(&s_max, lane_nc);
    __syncthreads();
    const int64_t end = start + (int64_t)s_max;
    const uint32_t wave_nc = wave_max_u32(lane_nc);
    const float kinv = -1.0f / kLog2e;
    unsigned long long n_eval = 0, n_blend = 0;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f, a6 = 0.f, a7 = 0.f, a8 = 0.f;
    for (int64_t base = start; base < end; base += CHUNK) {
        const int cnt = (int)min((int64_t)CHUNK, end - base);
        __syncthreads();  // the previous chunk's LDS is no longer read
        for (int k = threadIdx.x; k < cnt; k += NT) {
            const uint32_t gid = ids[base + k];
            s_gid[k] = gid;
            stage_splat(recs[gid], s_sp[k]);
        }
        __syncthreads();
        const uint32_t rel0 = (uint32_t)(base - start);
        // entries past this wave's last contributor need no work
        const int jend = wave_nc > rel0 ? (int)min((uint32_t)cnt, wave_nc - rel0) : 0;
        for (int j = 0; j < jend; ++j) {
            const Splat s = to_splat(s_sp[j]);
            float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f, e4 = 0.f, e5 = 0.f, e6 = 0.f, e7 = 0.f, e8 = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                float dx, dy, Gk, alpha;
                bool clamped;
                const bool live = rel0 + (uint32_t)j < nc[k];
                const bool ok = live && eval_splat(s, px[k], py[k], pxc[k], pyc[k], dx, dy, Gk, alpha, clamped);
                if (STATS) {
                    n_eval += (live && in_square(s, px[k], py[k])) ? 1u : 0u;
                    n_blend += ok ? 1u : 0u;
                }
                any = any || ok;
                const float w = ok ? alpha * T[k] : 0.0f;
                pr[k] = __builtin_fmaf(s.cr, w, pr[k]);
                pg[k] = __builtin_fmaf(s.cg, w, pg[k]);
                pb[k] = __builtin_fmaf(s.cb, w, pb[k]);
                // colour behind this splat: C_out - prefix (includes T_final * bg)
                const float oma = 1.0f - alpha;
                const float ioma = 1.0f / oma;
                const float Tk = T[k];
                const float da = G0[k] * (s.cr * Tk - (C0[k] - pr[k]) * ioma) +
                                 G1[k] * (s.cg * Tk - (C1[k] - pg[k]) * ioma) +
                                 G2[k] * (s.cb * Tk - (C2[k] - pb[k]) * ioma);
                e6 += G0[k] * w;
                e7 += G1[k] * w;
                e8 += G2[k] * w;
                const bool soft = ok && !clamped;
                const float dpn = soft ? da * alpha : 0.0f;  // dL/dpower (natural log domain)
                e5 += soft ? da * Gk : 0.0f;
                // power = -1/2 (Q00 dx^2 + 2 Q01 dx dy + Q11 dy^2); (qa, qb, qc) = log2(e) * (-Q00/2, -Q01, -Q11/2)
                const float kk = dpn * kinv;
                const float ddx = soft ? dx : 0.0f, ddy = soft ? dy : 0.0f;
                e0 += kk * (2.0f * s.qa * ddx + s.qb * ddy);  // dL/du
                e1 += kk * (s.qb * ddx + 2.0f * s.qc * ddy);  // dL/dv
                e2 += -0.5f * dpn * ddx * ddx;                // dL/dQ00
                e3 += -dpn * ddx * ddy;                       // dL/dQ01
                e4 += -0.5f * dpn * ddy * ddy;                // dL/dQ11
                T[k] = ok ? next_T(Tk, alpha) : Tk;
            }
            if (__ballot(any) != 0ull) {  // wave-uniform: reduce only when some lane blended
                // The reductions and the reads of lane 63 must run with the
                // whole wave active: the empty asm statement consumes the nine
                // wave sums here, so they cannot be moved into the lane-divergent
                // selects below that park them in lane j % 64.
                const int slot = j & 63;
                const int r0 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e0)), 63);
                const int r1 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e1)), 63);
                const int r2 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e2)), 63);
                const int r3 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e3)), 63);
                const int r4 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e4)), 63);
                const int r5 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e5)), 63);
                const int r6 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e6)), 63);
                const int r7 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e7)), 63);
                const int r8 = __builtin_amdgcn_readlane(__float_as_int(wave_sum_to_63(e8)), 63);
                asm volatile("" ::"s"(r0), "s"(r1), "s"(r2), "s"(r3), "s"(r4), "s"(r5), "s"(r6), "s"(r7), "s"(r8));
                const bool mine = lane == slot;
                a0 = mine ? __int_as_float(r0) : a0;
                a1 = mine ? __int_as_float(r1) : a1;
                a2 = mine ? __int_as_float(r2) : a2;
                a3 = mine ? __int_as_float(r3) : a3;
                a4 = mine ? __int_as_float(r4) : a4;
                a5 = mine ? __int_as_float(r5) : a5;
                a6 = mine ? __int_as_float(r6) : a6;
                a7 = mine ? __int_as_float(r7) : a7;
                a8 = mine ? __int_as_float(r8) : a8;
            }
            if ((j & 63) == 63 || j == jend - 1) {  // flush the group of up to 64 splats
                const int j0 = j & ~63;
                if (lane <= (j & 63)) {
                    const uint32_t gid = s_gid[j0 + lane];
                    if (a0 != 0.f) atomicAdd(&g2[(size_t)0 * N + gid], a0);
                    if (a1 != 0.f) atomicAdd(&g2[(size_t)1 * N + gid], a1);
                    if (a2 != 0.f) atomicAdd(&g2[(size_t)2 * N + gid], a2);
                    if (a3 != 0.f) atomicAdd(&g2[(size_t)3 * N + gid], a3);
                    if (a4 != 0.f) atomicAdd(&g2[(size_t)4 * N + gid], a4);
                    if (a5 != 0.f) atomicAdd(&g2[(size_t)5 * N + gid], a5);
                    if (a6 != 0.f) atomicAdd(&g2[(size_t)6 * N + gid], a6);
                    if (a7 != 0.f) atomicAdd(&g2[(size_t)7 * N + gid], a7);
                    if (a8 != 0.f) atomicAdd(&g2[(size_t)8 * N + gid], a8);
                }
                a0 = a1 = a2 = a3 = a4 = a5 = a6 = a7 = a8 = 0.f;
            }
        }
    }
    if (STATS) {
        atomicAdd(&counters[2], n_eval);
        atomicAdd(&counters[3], n_blend);
    }
}

bool composite_supported(int tile, int chunk) {
    return (tile == 8 || tile == 16 || tile == 32) && (chunk == 64 || chunk == 128 || chunk == 256 || chunk == 512);
}

template <int B, int C>
static void fwd_t(const Rec* recs, int N, const uint32_t* ids, const int64_t* ranges, const ViewParams* views, int v0,
                  int v1, int n_tiles, const PtrTable& images, float* Tfin, uint32_t* ncontrib, float* Cout,
                  unsigned long long* counters, hipStream_t st) {
    constexpr int NT = Shape<B>::NT;
    if (counters)
        k_composite_fwd<B, C, true><<<n_tiles, NT, 0, st>>>(recs, N, ids, ranges, views, v0, v1, images, Tfin,
                                                            ncontrib, Cout, counters);
    else
        k_composite_fwd<B, C, false><<<n_tiles, NT, 0, st>>>(recs, N, ids, ranges, views, v0, v1, images, Tfin,
                                                             ncontrib, Cout, nullptr);
}
template <int B, int C>
static void bwd_t(const Rec* recs, int N, const uint32_t* ids, const int64_t* ranges, const ViewParams* views, int v0,
                  int v1, int n_tiles, const CPtrTable& dls, const float* Tfin, const uint32_t* ncontrib,
                  const float* Cout, float* g2, unsigned long long* counters, hipStream_t st) {
    constexpr int NT = Shape<B>::NT;
    if (counters)
        k_composite_bwd<B, C, true><<<n_tiles, NT, 0, st>>>(recs, N, ids, ranges, views, v0, v1, dls, Tfin, ncontrib,
                                                            Cout, g2, counters);
    else
        k_composite_bwd<B, C, false><<<n_tiles, NT, 0, st>>>(recs, N, ids, ranges, views, v0, v1, dls, Tfin,
                                                             ncontrib, Cout, g2, nullptr);
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

void launch_composite_fwd(int tile, int chunk, const Rec* recs, int N, const uint32_t* ids, const int64_t* ranges,
                          const ViewParams* views, int v0, int v1, int n_tiles, const PtrTable& images, float* Tfin,
                          uint32_t* ncontrib, float* Cout, unsigned long long* counters, hipStream_t st) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(fwd_t, recs, N, ids, ranges, views, v0, v1, n_tiles, images, Tfin, ncontrib, Cout, counters, st);
}

void launch_composite_bwd(int tile, int chunk, const Rec* recs, int N, const uint32_t* ids, const int64_t* ranges,
                          const ViewParams* views, int v0, int v1, int n_tiles, const CPtrTable& dls,
                          const float* Tfin, const uint32_t* ncontrib, const float* Cout, float* g2,
                          unsigned long long* counters, hipStream_t st) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(bwd_t, recs, N, ids, ranges, views, v0, v1, n_tiles, dls, Tfin, ncontrib, Cout, g2, counters, st);
}

}  // namespace h4d

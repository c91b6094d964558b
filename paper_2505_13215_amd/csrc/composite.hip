// Front-to-back blending on gfx950 (Eq. 3; Alg. 1 BlendInOrder) and its adjoint.
//
// One workgroup per B x B tile, one lane per pixel (B = 8: one wave64; 16: four;
// 32: sixteen).  The tile's depth-ordered list is walked in chunks: each chunk of
// records is gathered once from HBM into LDS and broadcast to every lane.
// A pixel's contributors are exactly the splats whose pixel square contains it,
// so the image does not depend on B or on the chunk size.
//
// The backward recomputes transmittance front to back with the very same
// blending step as the forward (eval_splat), takes the colour behind a splat as
// C_out minus the running prefix, reduces the nine per-splat gradients across the
// wave with DPP, skips that when no lane of the wave blended the splat, adds the
// wave sums into LDS from one lane and flushes one global atomic per (splat,
// component, tile).  Each wave stops at its own last contributor.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

struct __align__(16) LSplat {
    int4 rect;     // x0, x1, y0, y1
    float4 pos;    // ui, uf, vi, vf
    float4 conic;  // qa, qb, qc, op
    float4 col;    // r, g, b, (unused)
};

__device__ __forceinline__ void stage_splat(const Rec& r, LSplat& s) {
    s.rect = make_int4((int)(r.d.x & 0xFFFFu), (int)(r.d.x >> 16), (int)(r.d.y & 0xFFFFu), (int)(r.d.y >> 16));
    s.pos = make_float4(r.c.y, r.a.x, r.c.z, r.a.y);
    s.conic = make_float4(r.a.z, r.a.w, r.b.x, r.b.y);
    s.col = make_float4(r.b.z, r.b.w, r.c.x, 0.f);
}

__device__ __forceinline__ Splat to_splat(const LSplat& l) {
    Splat s;
    s.x0 = l.rect.x; s.x1 = l.rect.y; s.y0 = l.rect.z; s.y1 = l.rect.w;
    s.ui = l.pos.x; s.uf = l.pos.y; s.vi = l.pos.z; s.vf = l.pos.w;
    s.qa = l.conic.x; s.qb = l.conic.y; s.qc = l.conic.z; s.op = l.conic.w;
    s.cr = l.col.x; s.cg = l.col.y; s.cb = l.col.z;
    return s;
}

__device__ __forceinline__ float next_T(float T, float alpha) {
#pragma clang fp contract(off)
    const float oma = 1.0f - alpha;
    return T * oma;
}

__device__ __forceinline__ bool in_square(const Splat& s, int px, int py) {
    return px >= s.x0 && px <= s.x1 && py >= s.y0 && py <= s.y1;
}

// STATS = true is a measurement-only instantiation that also counts (pixel,
// splat) evaluations and blends into counters[0..1].
template <int B, int CHUNK, bool STATS>
__global__ void __launch_bounds__(B * B) k_composite_fwd(const Rec* __restrict__ recs, const uint32_t* __restrict__ ids,
                                                         const int64_t* __restrict__ ranges,
                                                         const ViewParams* __restrict__ views, int view,
                                                         float* __restrict__ image, float* __restrict__ Tfin,
                                                         uint32_t* __restrict__ ncontrib, float* __restrict__ Cout,
                                                         unsigned long long* counters) {
    constexpr int NT = B * B;
    __shared__ LSplat s_sp[CHUNK];
    const ViewParams& V = views[view];
    const int tile = blockIdx.x;
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    const int px = tx * B + (int)(threadIdx.x % B), py = ty * B + (int)(threadIdx.x / B);
    const bool inside = px < V.W && py < V.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    const int64_t start = ranges[2 * (size_t)(V.tile_base + tile)];
    const int64_t end = ranges[2 * (size_t)(V.tile_base + tile) + 1];
    float T = 1.0f, cr = 0.f, cg = 0.f, cb = 0.f;
    uint32_t last = 0;
    unsigned long long n_eval = 0, n_blend = 0;
    bool done = !inside;
    for (int64_t base = start; base < end; base += CHUNK) {
        if (__syncthreads_count(done) == NT) break;
        const int cnt = (int)min((int64_t)CHUNK, end - base);
        for (int k = threadIdx.x; k < cnt; k += NT) stage_splat(recs[ids[base + k]], s_sp[k]);
        __syncthreads();
        if (!done) {
            for (int j = 0; j < cnt; ++j) {
                const Splat s = to_splat(s_sp[j]);
                float dx, dy, G, alpha;
                bool clamped;
                if (STATS && in_square(s, px, py)) ++n_eval;
                if (!eval_splat(s, px, py, pxc, pyc, dx, dy, G, alpha, clamped)) continue;
                const float Tn = next_T(T, alpha);
                if (Tn < kMinT) {
                    done = true;
                    break;
                }
                if (STATS) ++n_blend;
                const float w = alpha * T;
                cr = __builtin_fmaf(s.cr, w, cr);
                cg = __builtin_fmaf(s.cg, w, cg);
                cb = __builtin_fmaf(s.cb, w, cb);
                T = Tn;
                last = (uint32_t)(base - start) + (uint32_t)j + 1u;
            }
        }
    }
    if (inside) {
        const size_t HW = (size_t)V.W * V.H;
        const size_t p = (size_t)py * V.W + px;
        const float o0 = __builtin_fmaf(T, V.bg[0], cr), o1 = __builtin_fmaf(T, V.bg[1], cg),
                    o2 = __builtin_fmaf(T, V.bg[2], cb);
        image[p] = o0;
        image[HW + p] = o1;
        image[2 * HW + p] = o2;
        const size_t q = (size_t)V.pix_base + p;
        Tfin[q] = T;
        ncontrib[q] = last;
        Cout[3 * (size_t)V.pix_base + p] = o0;
        Cout[3 * (size_t)V.pix_base + HW + p] = o1;
        Cout[3 * (size_t)V.pix_base + 2 * HW + p] = o2;
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

template <int B, int CHUNK, bool STATS>
__global__ void __launch_bounds__(B * B) k_composite_bwd(const Rec* __restrict__ recs, const uint32_t* __restrict__ ids,
                                                         const int64_t* __restrict__ ranges,
                                                         const ViewParams* __restrict__ views, int view,
                                                         const float* __restrict__ dl, const float* __restrict__ Tfin,
                                                         const uint32_t* __restrict__ ncontrib,
                                                         const float* __restrict__ Cout, float* __restrict__ g2,
                                                         int N, unsigned long long* counters) {
    constexpr int NT = B * B;
    __shared__ LSplat s_sp[CHUNK];
    __shared__ uint32_t s_gid[CHUNK];
    // wave sums of the chunk's splats (one LDS atomic per wave and component);
    // a single slot keeps the block's LDS small and its occupancy high
    constexpr int NW = NT / 64;
    constexpr int SLOTS = 1;
    __shared__ float s_acc[SLOTS][9][CHUNK];
    __shared__ uint32_t s_max;
    const ViewParams& V = views[view];
    const int tile = blockIdx.x;
    const int tx = tile % V.tiles_x, ty = tile / V.tiles_x;
    const int px = tx * B + (int)(threadIdx.x % B), py = ty * B + (int)(threadIdx.x / B);
    const bool inside = px < V.W && py < V.H;
    const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
    const int64_t start = ranges[2 * (size_t)(V.tile_base + tile)];
    const size_t HW = (size_t)V.W * V.H;
    const size_t p = inside ? (size_t)py * V.W + px : 0;
    const size_t q = (size_t)V.pix_base + p;
    float G0 = 0.f, G1 = 0.f, G2 = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    uint32_t nc = 0;
    if (inside) {
        G0 = dl[p]; G1 = dl[HW + p]; G2 = dl[2 * HW + p];
        C0 = Cout[3 * (size_t)V.pix_base + p];
        C1 = Cout[3 * (size_t)V.pix_base + HW + p];
        C2 = Cout[3 * (size_t)V.pix_base + 2 * HW + p];
        nc = ncontrib[q];
    }
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    if (nc) atomicMax(&s_max, nc);
    __syncthreads();
    const int64_t end = start + (int64_t)s_max;
    const uint32_t wave_nc = wave_max_u32(nc);
    float T = 1.0f, pr = 0.f, pg = 0.f, pb = 0.f;
    const float kinv = -1.0f / kLog2e;
    unsigned long long n_eval = 0, n_blend = 0;
    for (int64_t base = start; base < end; base += CHUNK) {
        const int cnt = (int)min((int64_t)CHUNK, end - base);
        for (int k = threadIdx.x; k < cnt; k += NT) {
            const uint32_t gid = ids[base + k];
            s_gid[k] = gid;
            stage_splat(recs[gid], s_sp[k]);
        }
        for (int k = threadIdx.x; k < SLOTS * 9 * CHUNK; k += NT) (&s_acc[0][0][0])[k] = 0.f;
        __syncthreads();
        const uint32_t rel0 = (uint32_t)(base - start);
        // entries past this wave's last contributor need no work
        const int jend = wave_nc > rel0 ? (int)min((uint32_t)cnt, wave_nc - rel0) : 0;
        for (int j = 0; j < jend; ++j) {
            const Splat s = to_splat(s_sp[j]);
            float dx = 0.f, dy = 0.f, Gk = 0.f, alpha = 0.f;
            bool clamped = false;
            const bool bl = (rel0 + (uint32_t)j < nc) && eval_splat(s, px, py, pxc, pyc, dx, dy, Gk, alpha, clamped);
            if (STATS) {
                n_eval += (rel0 + (uint32_t)j < nc) && in_square(s, px, py);
                n_blend += bl;
            }
            if (__ballot(bl) == 0ull) continue;  // wave-uniform skip
            float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f, v6 = 0.f, v7 = 0.f, v8 = 0.f;
            if (bl) {
                const float w = alpha * T;
                pr = __builtin_fmaf(s.cr, w, pr);
                pg = __builtin_fmaf(s.cg, w, pg);
                pb = __builtin_fmaf(s.cb, w, pb);
                const float oma = 1.0f - alpha;
                const float ioma = 1.0f / oma;
                // colour behind this splat: C_out - prefix (includes T_final * bg)
                const float Sr = C0 - pr, Sg = C1 - pg, Sb = C2 - pb;
                const float da = G0 * (s.cr * T - Sr * ioma) + G1 * (s.cg * T - Sg * ioma) + G2 * (s.cb * T - Sb * ioma);
                v6 = G0 * w;
                v7 = G1 * w;
                v8 = G2 * w;
                if (!clamped) {
                    v5 = da * Gk;
                    const float dpn = da * alpha;  // dL/dpower (natural log domain)
                    // power = -1/2 (Q00 dx^2 + 2 Q01 dx dy + Q11 dy^2); (qa, qb, qc) = log2(e) * (-Q00/2, -Q01, -Q11/2)
                    const float kk = dpn * kinv;
                    v0 = kk * (2.0f * s.qa * dx + s.qb * dy);  // dL/du
                    v1 = kk * (s.qb * dx + 2.0f * s.qc * dy);  // dL/dv
                    v2 = -0.5f * dpn * dx * dx;                // dL/dQ00
                    v3 = -dpn * dx * dy;                       // dL/dQ01
                    v4 = -0.5f * dpn * dy * dy;                // dL/dQ11
                }
                T = next_T(T, alpha);
            }
            const float r0 = wave_sum_to_63(v0), r1 = wave_sum_to_63(v1), r2 = wave_sum_to_63(v2),
                        r3 = wave_sum_to_63(v3), r4 = wave_sum_to_63(v4), r5 = wave_sum_to_63(v5),
                        r6 = wave_sum_to_63(v6), r7 = wave_sum_to_63(v7), r8 = wave_sum_to_63(v8);
            if (__lane_id() == 63) {
                if (NW == 1) {
                    float* a = &s_acc[0][0][j];
                    a[0 * CHUNK] = r0; a[1 * CHUNK] = r1; a[2 * CHUNK] = r2;
                    a[3 * CHUNK] = r3; a[4 * CHUNK] = r4; a[5 * CHUNK] = r5;
                    a[6 * CHUNK] = r6; a[7 * CHUNK] = r7; a[8 * CHUNK] = r8;
                } else {
                    atomicAdd(&s_acc[0][0][j], r0); atomicAdd(&s_acc[0][1][j], r1);
                    atomicAdd(&s_acc[0][2][j], r2); atomicAdd(&s_acc[0][3][j], r3);
                    atomicAdd(&s_acc[0][4][j], r4); atomicAdd(&s_acc[0][5][j], r5);
                    atomicAdd(&s_acc[0][6][j], r6); atomicAdd(&s_acc[0][7][j], r7);
                    atomicAdd(&s_acc[0][8][j], r8);
                }
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < 9 * cnt; k += NT) {
            const int c = k / cnt, j = k - c * cnt;
            float val = s_acc[0][c][j];
            for (int w = 1; w < SLOTS; ++w) val += s_acc[w][c][j];
            if (val != 0.f) atomicAdd(&g2[(size_t)c * N + s_gid[j]], val);
        }
        __syncthreads();
    }
    if (STATS) {
        atomicAdd(&counters[2], n_eval);
        atomicAdd(&counters[3], n_blend);
    }
}

bool composite_supported(int tile, int chunk) {
    return (tile == 8 || tile == 16 || tile == 32) && (chunk == 128 || chunk == 256 || chunk == 512);
}

template <int B, int C>
static void fwd_t(const Rec* recs, const uint32_t* ids, const int64_t* ranges, const ViewParams* views, int view,
                  int n_tiles, float* image, float* Tfin, uint32_t* ncontrib, float* Cout, unsigned long long* counters,
                  hipStream_t st) {
    if (counters)
        k_composite_fwd<B, C, true><<<n_tiles, B * B, 0, st>>>(recs, ids, ranges, views, view, image, Tfin, ncontrib,
                                                               Cout, counters);
    else
        k_composite_fwd<B, C, false><<<n_tiles, B * B, 0, st>>>(recs, ids, ranges, views, view, image, Tfin, ncontrib,
                                                                Cout, nullptr);
}
template <int B, int C>
static void bwd_t(const Rec* recs, const uint32_t* ids, const int64_t* ranges, const ViewParams* views, int view,
                  int n_tiles, const float* dl, const float* Tfin, const uint32_t* ncontrib, const float* Cout,
                  float* g2, int N, unsigned long long* counters, hipStream_t st) {
    if (counters)
        k_composite_bwd<B, C, true><<<n_tiles, B * B, 0, st>>>(recs, ids, ranges, views, view, dl, Tfin, ncontrib, Cout,
                                                               g2, N, counters);
    else
        k_composite_bwd<B, C, false><<<n_tiles, B * B, 0, st>>>(recs, ids, ranges, views, view, dl, Tfin, ncontrib,
                                                                Cout, g2, N, nullptr);
}

#define H4D_DISPATCH(FN, ...)                                                   \
    do {                                                                        \
        if (tile == 8 && chunk == 128) FN<8, 128>(__VA_ARGS__);                 \
        else if (tile == 8 && chunk == 256) FN<8, 256>(__VA_ARGS__);            \
        else if (tile == 8 && chunk == 512) FN<8, 512>(__VA_ARGS__);            \
        else if (tile == 16 && chunk == 128) FN<16, 128>(__VA_ARGS__);          \
        else if (tile == 16 && chunk == 256) FN<16, 256>(__VA_ARGS__);          \
        else if (tile == 16 && chunk == 512) FN<16, 512>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 128) FN<32, 128>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 256) FN<32, 256>(__VA_ARGS__);          \
        else if (tile == 32 && chunk == 512) FN<32, 512>(__VA_ARGS__);          \
    } while (0)

void launch_composite_fwd(int tile, int chunk, const Rec* recs, const uint32_t* ids, const int64_t* ranges,
                          const ViewParams* views, int view, int n_tiles, float* image, float* Tfin,
                          uint32_t* ncontrib, float* Cout, unsigned long long* counters, hipStream_t st) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(fwd_t, recs, ids, ranges, views, view, n_tiles, image, Tfin, ncontrib, Cout, counters, st);
}

void launch_composite_bwd(int tile, int chunk, const Rec* recs, const uint32_t* ids, const int64_t* ranges,
                          const ViewParams* views, int view, int n_tiles, const float* dl, const float* Tfin,
                          const uint32_t* ncontrib, const float* Cout, float* g2, int N, unsigned long long* counters,
                          hipStream_t st) {
    if (n_tiles == 0) return;
    H4D_DISPATCH(bwd_t, recs, ids, ranges, views, view, n_tiles, dl, Tfin, ncontrib, Cout, g2, N, counters, st);
}

}  // namespace h4d

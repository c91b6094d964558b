// Host-side check of the binning's tabulated tile spans (built and run by
// test_binning_spans.py; no GPU is used).  For random splats (covariances,
// opacities, centres on and off the image, pixel squares as the projection
// computes them) it compares, for every super-tile of the splat's square, the
// tile mask of the per-entry ellipse test (tile_mask with culling) with the
// mask the emission builds from the count kernel's output: the rectangle
// shrunk to the slab rows and the spans' columns (slab_rows, row_span), the
// spans (span_mask), or, for splats taller than the table, the per-entry test
// on the shrunk rectangle.  Prints "mismatches M entries E0 E1" per tile size.
#include "../paper_2505_13215_amd/csrc/sort.hip"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>

using namespace h4d;

template <int TILE>
static void check(std::mt19937_64& rng, int splats) {
    constexpr uint32_t S = super_factor(TILE);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long mismatches = 0, entries_square = 0, entries_shrunk = 0;
    for (int it = 0; it < splats; ++it) {
        const int W = 640 + (int)(U(rng) * 2100), H = 480 + (int)(U(rng) * 1600);
        const double u = -80.0 + U(rng) * (W + 160), v = -80.0 + U(rng) * (H + 160);
        // covariance eigenvalues from 0.05 to 400 px^2 (to 40000 for 5 %), any
        // orientation, anisotropy up to 1000
        const double hi = U(rng) < 0.05 ? 40000.0 : 400.0;
        const double l1 = std::exp(std::log(0.05) + U(rng) * (std::log(hi) - std::log(0.05)));
        const double l2 = l1 * std::exp(std::log(1e-3) * U(rng));
        const double th = U(rng) * 3.141592653589793, c = std::cos(th), s = std::sin(th);
        const double sa = c * c * l1 + s * s * l2 + 0.3, sb = c * s * (l1 - l2), sc = s * s * l1 + c * c * l2 + 0.3;
        const double det = sa * sc - sb * sb;
        const double qa = sc / det, qb = -sb / det, qc = sa / det, k = -0.5 * 1.4426950408889634;
        const double lam = 0.5 * (sa + sc) + std::sqrt(0.25 * (sa - sc) * (sa - sc) + sb * sb);
        const int r = (int)std::ceil(3.0 * std::sqrt(lam));
        const int x0 = std::max(0, (int)std::ceil(u - r - 0.5)), x1 = std::min(W - 1, (int)std::floor(u + r - 0.5));
        const int y0 = std::max(0, (int)std::ceil(v - r - 0.5)), y1 = std::min(H - 1, (int)std::floor(v + r - 0.5));
        if (x0 > x1 || y0 > y1) continue;
        const double op = U(rng) < 0.1 ? 0.01 * U(rng) : U(rng);
        Rec rec;
        const double fu = std::floor(u), fv = std::floor(v);
        rec.a = make_float4((float)(u - fu), (float)(v - fv), (float)(qa * k), (float)(qb * 2.0 * k));
        rec.b = make_float4((float)(qc * k), (float)op, 0.f, 0.f);
        rec.c = make_float4(0.f, (float)fu, (float)fv, 1.f);
        rec.d = make_uint4((uint32_t)x0 | ((uint32_t)x1 << 16), (uint32_t)y0 | ((uint32_t)y1 << 16), (uint32_t)r, 1u);
        const CullShape cs = cull_shape(rec);
        const uint32_t tx0 = x0 / TILE, tx1 = x1 / TILE, ty0 = y0 / TILE, ty1 = y1 / TILE;
        // the count kernel's rectangle and spans, one splat at a time
        bool keep = cs.mode != 2;
        bool full = cs.mode == 0, table = true;
        uint32_t nx0 = tx0, nx1 = tx1, ny0 = ty0, ny1 = ty1, spans[kSpanRows];
        if (cs.mode == 1) {
            int r0, r1;
            slab_rows<TILE>(cs, (int)ty0, (int)ty1, r0, r1);
            table = r1 - r0 < kSpanRows;
            int cmin = (int)tx1 + 1, cmax = (int)tx0 - 1;
            for (int ty = r0; ty <= r1; ++ty) {
                const uint32_t e = row_span<TILE>(cs, ty, (int)tx0, (int)tx1);
                if (table) spans[ty - r0] = e;
                if (e != 0u) {
                    cmin = std::min(cmin, (int)(e & 0xFFFFu));
                    cmax = std::max(cmax, (int)(e >> 16) - 1);
                }
            }
            keep = cmin <= cmax;
            nx0 = (uint32_t)cmin; nx1 = (uint32_t)cmax; ny0 = (uint32_t)r0; ny1 = (uint32_t)r1;
        }
        for (uint32_t sy = ty0 / S; sy <= ty1 / S; ++sy)
            for (uint32_t sx = tx0 / S; sx <= tx1 / S; ++sx) {
                const uint32_t bx = sx * S, by = sy * S;
                const uint32_t m0 = cs.mode == 2 ? 0u : tile_mask<TILE>(cs, cs.mode == 1, tx0, tx1, ty0, ty1, bx, by);
                ++entries_square;
                uint32_t m1 = 0u;
                if (keep && sx >= nx0 / S && sx <= nx1 / S && sy >= ny0 / S && sy <= ny1 / S) {
                    ++entries_shrunk;
                    if (full) m1 = tile_mask<TILE>(cs, false, nx0, nx1, ny0, ny1, bx, by);
                    else if (!table) m1 = tile_mask<TILE>(cs, true, nx0, nx1, ny0, ny1, bx, by);
                    else m1 = span_mask<TILE>(spans, ny0, ny1, bx, by);
                }
                if (m0 != m1) ++mismatches;
            }
    }
    std::printf("tile %d mismatches %ld entries %ld %ld\n", TILE, mismatches, entries_square, entries_shrunk);
}

int main(int argc, char** argv) {
    const int splats = argc > 1 ? std::atoi(argv[1]) : 100000;
    std::mt19937_64 rng(20250513);
    check<8>(rng, splats);
    check<16>(rng, splats);
    check<32>(rng, splats);
    return 0;
}

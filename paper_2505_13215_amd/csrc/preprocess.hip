// Per-Gaussian stages of the rasterizer on gfx950, forward and backward:
// activations, covariance (Eq. 2, Eq. 4), slicing of 4D Gaussians at t (Eq. 5-6)
// with the temporal marginal opacity, culling, EWA projection, SH colour and
// the screen-space record that the binning and blending kernels consume.
//
// Geometry runs in FP64: CDNA4 issues FP64 vector FMAs at the FP32 (non-packed)
// rate, the stage is bound by its 236-260 B/Gaussian of parameter reads, and in
// FP64 every discrete decision of the stage (cull, radius, pixel square, depth
// key) lands exactly where the FP64 definition puts it.
#include "common.hpp"
#include "launch.hpp"
#include "rotation.hpp"

namespace h4d {

// ---------------------------------------------------------------------------
// Real SH basis of degree 3 (Condon-Shortley phase), evaluated as polynomials of
// the unit viewing direction, and its gradient.
// ---------------------------------------------------------------------------
namespace sh {
constexpr double C0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double C1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double C4 = 1.0925484305920792;    // sqrt(15/pi)/2
constexpr double C6 = 0.31539156525252005;   // sqrt(5/pi)/4
constexpr double C8 = 0.5462742152960396;    // sqrt(15/pi)/4
constexpr double C9 = 0.5900435899266435;    // sqrt(35/(2 pi))/4
constexpr double C10 = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double C11 = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double C12 = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double C14 = 1.445305721320277;    // sqrt(105/pi)/4
}  // namespace sh

__device__ inline void sh_eval(double x, double y, double z, double Y[16]) {
    using namespace sh;
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = C0;
    Y[1] = -C1 * y;
    Y[2] = C1 * z;
    Y[3] = -C1 * x;
    Y[4] = C4 * x * y;
    Y[5] = -C4 * y * z;
    Y[6] = C6 * (2.0 * zz - xx - yy);
    Y[7] = -C4 * x * z;
    Y[8] = C8 * (xx - yy);
    Y[9] = -C9 * y * (3.0 * xx - yy);
    Y[10] = C10 * x * y * z;
    Y[11] = -C11 * y * (4.0 * zz - xx - yy);
    Y[12] = C12 * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -C11 * x * (4.0 * zz - xx - yy);
    Y[14] = C14 * z * (xx - yy);
    Y[15] = -C9 * x * (xx - 3.0 * yy);
}

// w . dY/d(x,y,z) for a weight vector w[16] over the basis
__device__ inline void sh_grad_dot(double x, double y, double z, const double w[16], double g[3]) {
    using namespace sh;
    const double xx = x * x, yy = y * y, zz = z * z;
    double gx = 0, gy = 0, gz = 0;
    gy += w[1] * (-C1);
    gz += w[2] * C1;
    gx += w[3] * (-C1);
    gx += w[4] * C4 * y;            gy += w[4] * C4 * x;
    gy += w[5] * (-C4 * z);         gz += w[5] * (-C4 * y);
    gx += w[6] * (-2.0 * C6 * x);   gy += w[6] * (-2.0 * C6 * y);  gz += w[6] * (4.0 * C6 * z);
    gx += w[7] * (-C4 * z);         gz += w[7] * (-C4 * x);
    gx += w[8] * (2.0 * C8 * x);    gy += w[8] * (-2.0 * C8 * y);
    gx += w[9] * (-6.0 * C9 * x * y);              gy += w[9] * (-C9 * (3.0 * xx - 3.0 * yy));
    gx += w[10] * C10 * y * z;      gy += w[10] * C10 * x * z;     gz += w[10] * C10 * x * y;
    gx += w[11] * (2.0 * C11 * x * y);             gy += w[11] * (-C11 * (4.0 * zz - xx - 3.0 * yy));
    gz += w[11] * (-8.0 * C11 * y * z);
    gx += w[12] * (-6.0 * C12 * x * z);            gy += w[12] * (-6.0 * C12 * y * z);
    gz += w[12] * (C12 * (6.0 * zz - 3.0 * xx - 3.0 * yy));
    gx += w[13] * (-C11 * (4.0 * zz - 3.0 * xx - yy)); gy += w[13] * (2.0 * C11 * x * y);
    gz += w[13] * (-8.0 * C11 * x * z);
    gx += w[14] * (2.0 * C14 * x * z);             gy += w[14] * (-2.0 * C14 * y * z);
    gz += w[14] * (C14 * (xx - yy));
    gx += w[15] * (-C9 * (3.0 * xx - 3.0 * yy));   gy += w[15] * (6.0 * C9 * x * y);
    g[0] = gx; g[1] = gy; g[2] = gz;
}

// ---------------------------------------------------------------------------
// World stage (view independent except for the timestamp of a 4D Gaussian).
// ---------------------------------------------------------------------------
struct WorldF {
    double mu[3];
    double S[3][3];  // covariance at time t
    double op;       // sigmoid(o) * p(t)
};

struct Rot4 {
    double L[4][4], Rr[4][4], R[4][4];
};

__device__ inline double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

// 4D Gaussian i at time t.  Fills the 4D intermediates the adjoint needs.
struct Slice4 {
    double s[4], ql[4], qr[4], nl, nr;
    Rot4 rot;
    double S4[4][4];
    double b[3], c, delta, pt, sig;
};

__device__ inline void world4(const G4Ptr& g, int i, double time, WorldF& w, Slice4& z) {
    const int n = g.n;
    for (int k = 0; k < 4; ++k) z.s[k] = exp((double)g.log_scale[(size_t)k * n + i]);
    z.nl = load_unit4(g.quat_l, n, i, z.ql);
    z.nr = load_unit4(g.quat_r, n, i, z.qr);
    rot_left(z.ql, z.rot.L);
    rot_right(z.qr, z.rot.Rr);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0;
            for (int k = 0; k < 4; ++k) acc += z.rot.L[r][k] * z.rot.Rr[k][c];
            z.rot.R[r][c] = acc;
        }
    double s2[4];
    for (int k = 0; k < 4; ++k) s2[k] = z.s[k] * z.s[k];
    for (int r = 0; r < 4; ++r)
        for (int c = r; c < 4; ++c) {
            double acc = 0;
            for (int k = 0; k < 4; ++k) acc += z.rot.R[r][k] * s2[k] * z.rot.R[c][k];
            z.S4[r][c] = acc;
            z.S4[c][r] = acc;
        }
    // Eq. 5-6: condition the spatial block on time
    z.c = z.S4[3][3];
    z.delta = time - (double)g.mean_t[i];
    const double ic = 1.0 / z.c;
    for (int k = 0; k < 3; ++k) z.b[k] = z.S4[k][3];
    for (int k = 0; k < 3; ++k) w.mu[k] = (double)g.mean[(size_t)k * n + i] + z.b[k] * ic * z.delta;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) w.S[r][c] = z.S4[r][c] - z.b[r] * z.b[c] * ic;
    z.pt = exp(-(z.delta * z.delta) * 0.5 * ic);
    z.sig = sigmoid((double)g.opacity[i]);
    w.op = z.sig * z.pt;
}

struct Cov3 {
    double s[3], q[4], nq, R[3][3], sig;
};

__device__ inline void world3(const G3Ptr& g, int i, WorldF& w, Cov3& z) {
    const int n = g.n;
    for (int k = 0; k < 3; ++k) z.s[k] = exp((double)g.log_scale[(size_t)k * n + i]);
    z.nq = load_unit4(g.quat, n, i, z.q);
    quat_rot3(z.q, z.R);
    for (int r = 0; r < 3; ++r)
        for (int c = r; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += z.R[r][k] * z.s[k] * z.s[k] * z.R[c][k];
            w.S[r][c] = acc;
            w.S[c][r] = acc;
        }
    for (int k = 0; k < 3; ++k) w.mu[k] = (double)g.mean[(size_t)k * n + i];
    z.sig = sigmoid((double)g.opacity[i]);
    w.op = z.sig;
}

// ---------------------------------------------------------------------------
// Projection stage.
// ---------------------------------------------------------------------------
struct ProjF {
    bool culled, covered;
    double pc[3], x, y, xt, yt;
    bool clx, cly;
    double M[2][3];
    double a, b, d, det;
    double u, v;
    int r, x0, x1, y0, y1;
    double dir[3], en;
};

__device__ inline void project(const ViewParams& V, const WorldF& w, ProjF& p) {
    p.culled = true;
    p.covered = false;
    for (int i = 0; i < 3; ++i)
        p.pc[i] = V.R[3 * i] * w.mu[0] + V.R[3 * i + 1] * w.mu[1] + V.R[3 * i + 2] * w.mu[2] + V.T[i];
    if (p.pc[2] <= kNear || w.op < kMinAlphaD) return;
    const double iz = 1.0 / p.pc[2];
    p.x = p.pc[0] * iz;
    p.y = p.pc[1] * iz;
    const double limx = kClampFov * (0.5 * V.W / V.fx), limy = kClampFov * (0.5 * V.H / V.fy);
    p.clx = p.x > limx || p.x < -limx;
    p.cly = p.y > limy || p.y < -limy;
    p.xt = fmin(fmax(p.x, -limx), limx);
    p.yt = fmin(fmax(p.y, -limy), limy);
    const double J00 = V.fx * iz, J02 = -V.fx * p.xt * iz, J11 = V.fy * iz, J12 = -V.fy * p.yt * iz;
    for (int j = 0; j < 3; ++j) {
        p.M[0][j] = J00 * V.R[j] + J02 * V.R[6 + j];
        p.M[1][j] = J11 * V.R[3 + j] + J12 * V.R[6 + j];
    }
    // 2D covariance M S M^T (+ dilation)
    double MS[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) MS[r][c] = p.M[r][0] * w.S[0][c] + p.M[r][1] * w.S[1][c] + p.M[r][2] * w.S[2][c];
    p.a = MS[0][0] * p.M[0][0] + MS[0][1] * p.M[0][1] + MS[0][2] * p.M[0][2] + kDilate;
    p.b = MS[0][0] * p.M[1][0] + MS[0][1] * p.M[1][1] + MS[0][2] * p.M[1][2];
    p.d = MS[1][0] * p.M[1][0] + MS[1][1] * p.M[1][1] + MS[1][2] * p.M[1][2] + kDilate;
    p.det = p.a * p.d - p.b * p.b;
    if (p.det <= 0.0) return;
    const double mid = 0.5 * (p.a + p.d);
    const double lam = mid + sqrt(fmax(kEigFloor, mid * mid - p.det));
    p.r = (int)ceil(kSigmas * sqrt(lam));
    p.u = V.fx * p.x + V.cx;
    p.v = V.fy * p.y + V.cy;
    // pixel square |i + 0.5 - u| <= r, clipped to the image
    p.x0 = max(0, (int)ceil(p.u - p.r - 0.5));
    p.x1 = min(V.W - 1, (int)floor(p.u + p.r - 0.5));
    p.y0 = max(0, (int)ceil(p.v - p.r - 0.5));
    p.y1 = min(V.H - 1, (int)floor(p.v + p.r - 0.5));
    p.culled = false;
    p.covered = p.x0 <= p.x1 && p.y0 <= p.y1;
    double e[3] = {w.mu[0] - V.campos[0], w.mu[1] - V.campos[1], w.mu[2] - V.campos[2]};
    p.en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double ie = 1.0 / p.en;
    for (int k = 0; k < 3; ++k) p.dir[k] = e[k] * ie;
}

// raw (unclamped) colour of channel ch: 0.5 + sum_k sh[k][ch] Y_k
__device__ inline void colour(const float* shp, int n, int i, const double Y[16], double raw[3]) {
    for (int ch = 0; ch < 3; ++ch) {
        double acc = kShOffset;
        for (int k = 0; k < 16; ++k) acc += (double)shp[(size_t)(k * 3 + ch) * n + i] * Y[k];
        raw[ch] = acc;
    }
}

// Time weights of a 4D Gaussian's colour at view time t: w[k] = cos(2 pi (k +
// 1) (t - mean_t) / T) and their derivatives dw[k] with respect to mean_t.
__device__ inline void time_weights(const G4Ptr& g, int i, double time, double w[kMaxTimeDeg],
                                    double dw[kMaxTimeDeg]) {
    const double d = time - (double)g.mean_t[i];
    for (int k = 0; k < g.sh_t_deg; ++k) {
        const double om = 2.0 * M_PI * (double)(k + 1) / (double)g.sh_t_period;
        w[k] = cos(om * d);
        dw[k] = om * sin(om * d);
    }
}

// SH coefficient j of 4D Gaussian i at the time of the weights w.
__device__ inline double coef_at(const G4Ptr& g, int i, int j, const double w[kMaxTimeDeg]) {
    const size_t n = (size_t)g.n;
    double c = (double)g.sh[(size_t)j * n + i];
    for (int k = 0; k < g.sh_t_deg; ++k) c += w[k] * (double)g.sh_t[((size_t)k * 48 + j) * n + i];
    return c;
}

// Time coefficients of a 4D Gaussian's colour in the adjoint (null: none):
// weights and their mean_t derivatives at the view's time, the set, and the
// gradient rows (accumulated) of sh_t.
struct TimeColour {
    const G4Ptr* g;
    int i;
    double w[kMaxTimeDeg], dw[kMaxTimeDeg];
    float* gsht;
};

// ---------------------------------------------------------------------------
// Forward kernel: one thread per Gaussian of the merged list [4D | 3D].
// ---------------------------------------------------------------------------
// grid.y runs over the views [v0, v0 + gridDim.y): records go to recs[view][N]
// (absolute), depth keys and ids to the pass's segment layout: unshared,
// dkeys/dvals[view - v0][N]; shared (static binning per camera), the view's 4D
// Gaussians at (view - v0) n4 + g and, for a static group's leader view only,
// the 3D Gaussians at nv n4 + group n3 + (g - n4) (the other views of the group
// use the leader's 3D records and compute none).
// g2 (may be null): the screen-space gradient records, zeroed for the records
// that cover a pixel.
__global__ void __launch_bounds__(256) k_preprocess(G3Ptr g3, G4Ptr g4, const ViewParams* __restrict__ views,
                                                    int v0, int shared, Rec* __restrict__ recs,
                                                    uint32_t* __restrict__ dkeys, uint32_t* __restrict__ dvals,
                                                    float* __restrict__ g2) {
    const int N = g3.n + g4.n;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const int view = v0 + (int)blockIdx.y;
    const ViewParams& V = views[view];
    size_t slot;
    if (!shared) {
        slot = (size_t)blockIdx.y * N + g;
    } else if (g < g4.n) {
        slot = (size_t)blockIdx.y * g4.n + g;
    } else {
        if (V.static_view != view) return;  // the group's leader holds this 3D record
        slot = (size_t)gridDim.y * g4.n + (size_t)V.static_group * g3.n + (g - g4.n);
    }
    recs += (size_t)view * N;
    dkeys += slot - g;
    dvals += slot - g;
    WorldF w;
    const float* shp;
    int shn, shi;
    if (g < g4.n) {
        Slice4 z;
        world4(g4, g, V.time, w, z);
        shp = g4.sh; shn = g4.n; shi = g;
    } else {
        Cov3 z;
        world3(g3, g - g4.n, w, z);
        shp = g3.sh; shn = g3.n; shi = g - g4.n;
    }
    ProjF p;
    project(V, w, p);
    Rec rec;
    uint32_t key = kCulledKey;
    if (!p.culled && p.covered) {
        const double iD = 1.0 / p.det;
        const double Qa = p.d * iD, Qb = -p.b * iD, Qc = p.a * iD;
        const double s = -0.5 * 1.4426950408889634;  // -log2(e)/2
        double Y[16], raw[3];
        sh_eval(p.dir[0], p.dir[1], p.dir[2], Y);
        if (g < g4.n && g4.sh_t_deg > 0) {
            double tw[kMaxTimeDeg], tdw[kMaxTimeDeg];
            time_weights(g4, g, V.time, tw, tdw);
            for (int ch = 0; ch < 3; ++ch) {
                double acc = kShOffset;
                for (int k = 0; k < 16; ++k) acc += coef_at(g4, g, k * 3 + ch, tw) * Y[k];
                raw[ch] = acc;
            }
        } else {
            colour(shp, shn, shi, Y, raw);
        }
        const double fu = floor(p.u), fv = floor(p.v);
        rec.a = make_float4((float)(p.u - fu), (float)(p.v - fv), (float)(Qa * s), (float)(Qb * 2.0 * s));
        rec.b = make_float4((float)(Qc * s), (float)w.op, (float)fmax(raw[0], 0.0), (float)fmax(raw[1], 0.0));
        const float depth = (float)p.pc[2];
        rec.c = make_float4((float)fmax(raw[2], 0.0), (float)fu, (float)fv, depth);
        rec.d = make_uint4((uint32_t)p.x0 | ((uint32_t)p.x1 << 16), (uint32_t)p.y0 | ((uint32_t)p.y1 << 16),
                           (uint32_t)p.r, 1u);
        key = __float_as_uint(depth);
        if (g2) {
            float4* row = reinterpret_cast<float4*>(g2 + ((size_t)view * N + g) * kG2Stride);
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            row[0] = z;
            row[1] = z;
            row[2] = z;
            row[3] = z;
        }
    } else {
        rec.a = make_float4(0.f, 0.f, 0.f, 0.f);
        rec.b = rec.a;
        rec.c = rec.a;
        rec.d = make_uint4(0u, 0u, 0u, 0u);
    }
    recs[g] = rec;
    dkeys[g] = key;
    dvals[g] = (uint32_t)g;
}

// ---------------------------------------------------------------------------
// Backward kernel: one thread per Gaussian, looping over the views of the call
// (no atomics: every view's contribution to a Gaussian lands in one lane).
// g2: per (view, Gaussian) screen-space gradients from the blending adjoint,
// layout [view][N][kG2Stride]: du dv dQ00 dQ01 dQ11 dop dr dg, then db as
// four parts (w.r.t. the unscaled conic entries, Q01 counted once; the first
// five without their factors -op / log2 e, -op / log2 e, -op / 2, -op, -op / 2).
//
// Per view the projection adjoint gives mu_c-bar, Sigma_c-bar and op-bar; the
// slicing adjoint maps them to the spatial/temporal means and to the symmetric
// part of Sigma4-bar, which is summed over views so that the covariance and
// rotation adjoints run once per Gaussian.
// ---------------------------------------------------------------------------
// TIME: tc holds the Gaussian's time coefficients; their gradient rows are
// accumulated and gmt receives mean_t's share through the time weights (a
// separate instantiation, so that sets without them compile as plain SH).
template <bool TIME>
__device__ inline void proj_bwd(const ViewParams& V, const WorldF& w, const ProjF& p, const float* shp, int shn,
                                int shi, const float* g2, size_t gstride, double gmu[3], double Sb[3][3],
                                double& gop, float* gsh, const TimeColour* tc = nullptr, double* gmt = nullptr) {
    // the blending adjoint sums the centre and conic terms without their
    // constant factors and the effective opacity: du, dv take -op / log2 e,
    // dQ00, dQ11 -op / 2, dQ01 -op
    const double ku = -kLn2 * w.op, kq = -0.5 * w.op;
    const double gu = ku * g2[0], gv = ku * g2[gstride], gQa = kq * g2[2 * gstride], gQb = -w.op * g2[3 * gstride],
                 gQc = kq * g2[4 * gstride];
    gop = g2[5 * gstride];
    const double grgb[3] = {g2[6 * gstride], g2[7 * gstride],
                            (double)g2[8 * gstride] + g2[9 * gstride] + g2[10 * gstride] + g2[11 * gstride]};
    // colour
    double Y[16], raw[3];
    sh_eval(p.dir[0], p.dir[1], p.dir[2], Y);
    auto cf = [&](int j) {
        if constexpr (TIME) return coef_at(*tc->g, tc->i, j, tc->w);
        else return (double)shp[(size_t)j * shn + shi];
    };
    for (int ch = 0; ch < 3; ++ch) {
        double acc = kShOffset;
        for (int k = 0; k < 16; ++k) acc += cf(k * 3 + ch) * Y[k];
        raw[ch] = acc;
    }
    double gc[3];
    for (int ch = 0; ch < 3; ++ch) gc[ch] = raw[ch] > 0.0 ? grgb[ch] : 0.0;
    double wY[16];
    for (int k = 0; k < 16; ++k) {
        double acc = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
            gsh[k * 3 + ch] += (float)(gc[ch] * Y[k]);
            acc += gc[ch] * cf(k * 3 + ch);
        }
        wY[k] = acc;
    }
    if constexpr (TIME) {
        // dc_j / dsh_t[k][j] = w[k], dc_j / dmean_t = sum_k dw[k] sh_t[k][j]
        const size_t n = (size_t)tc->g->n;
        double gm = 0.0;
        for (int kk = 0; kk < tc->g->sh_t_deg; ++kk)
            for (int j = 0; j < 48; ++j) {
                const double gj = gc[j % 3] * Y[j / 3];
                const size_t o = ((size_t)kk * 48 + j) * n + tc->i;
                tc->gsht[o] += (float)(tc->w[kk] * gj);
                gm += gj * tc->dw[kk] * (double)tc->g->sh_t[o];
            }
        *gmt += gm;
    }
    double gd[3];
    sh_grad_dot(p.dir[0], p.dir[1], p.dir[2], wY, gd);
    const double dd = p.dir[0] * gd[0] + p.dir[1] * gd[1] + p.dir[2] * gd[2];
    const double ie = 1.0 / p.en;
    for (int k = 0; k < 3; ++k) gmu[k] = (gd[k] - p.dir[k] * dd) * ie;
    // conic -> 2D covariance: S2bar = -Q Gbar Q, Gbar = [[gQa, gQb/2], [gQb/2, gQc]]
    const double iD = 1.0 / p.det;
    const double Q00 = p.d * iD, Q01 = -p.b * iD, Q11 = p.a * iD;
    const double G00 = gQa, G01 = 0.5 * gQb, G11 = gQc;
    const double T00 = Q00 * G00 + Q01 * G01, T01 = Q00 * G01 + Q01 * G11;
    const double T10 = Q01 * G00 + Q11 * G01, T11 = Q01 * G01 + Q11 * G11;
    const double B00 = -(T00 * Q00 + T01 * Q01), B01 = -(T00 * Q01 + T01 * Q11);
    const double B11 = -(T10 * Q01 + T11 * Q11);
    // Sigma_c bar = M^T B M (symmetric)
    double BM[2][3];
    for (int c = 0; c < 3; ++c) {
        BM[0][c] = B00 * p.M[0][c] + B01 * p.M[1][c];
        BM[1][c] = B01 * p.M[0][c] + B11 * p.M[1][c];
    }
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const double v = p.M[0][i] * BM[0][j] + p.M[1][i] * BM[1][j];
            Sb[i][j] = v;
            Sb[j][i] = v;
        }
    // M bar = 2 B M Sigma_c ; J bar = M bar R^T (only the four non-zero J entries matter)
    double Mb[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            Mb[r][c] = 2.0 * (BM[r][0] * w.S[0][c] + BM[r][1] * w.S[1][c] + BM[r][2] * w.S[2][c]);
    const double Jb00 = Mb[0][0] * V.R[0] + Mb[0][1] * V.R[1] + Mb[0][2] * V.R[2];
    const double Jb02 = Mb[0][0] * V.R[6] + Mb[0][1] * V.R[7] + Mb[0][2] * V.R[8];
    const double Jb11 = Mb[1][0] * V.R[3] + Mb[1][1] * V.R[4] + Mb[1][2] * V.R[5];
    const double Jb12 = Mb[1][0] * V.R[6] + Mb[1][1] * V.R[7] + Mb[1][2] * V.R[8];
    const double z = p.pc[2], iz = 1.0 / z, iz2 = iz * iz;
    double pb0, pb1, pb2;
    pb2 = -Jb00 * V.fx * iz2 + Jb02 * V.fx * p.xt * iz2 - Jb11 * V.fy * iz2 + Jb12 * V.fy * p.yt * iz2;
    double xb = gu * V.fx, yb = gv * V.fy;
    if (!p.clx) xb += -Jb02 * V.fx * iz;
    if (!p.cly) yb += -Jb12 * V.fy * iz;
    pb0 = xb * iz;
    pb1 = yb * iz;
    pb2 += -(xb * p.pc[0] + yb * p.pc[1]) * iz2;
    for (int k = 0; k < 3; ++k) gmu[k] += V.R[k] * pb0 + V.R[3 + k] * pb1 + V.R[6 + k] * pb2;
}

__device__ inline void unit_bwd(const double qh[4], double nrm, const double gqh[4], float* out, size_t stride) {
    const double dq = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
    const double in = 1.0 / nrm;
    for (int k = 0; k < 4; ++k) out[k * stride] = (float)((gqh[k] - qh[k] * dq) * in);
}

template <bool TIME>
__device__ inline void bwd_4d(const G4Ptr& g4, int i, const ViewParams* __restrict__ views, int n_views, int N,
                              const Rec* __restrict__ recs, const float* __restrict__ g2, const G4Grad& gr,
                              const SetStats& st) {
    const size_t n = (size_t)g4.n;
    double s[4], ql[4], qr[4];
    for (int k = 0; k < 4; ++k) s[k] = exp((double)g4.log_scale[k * n + i]);
    const double nl = load_unit4(g4.quat_l, g4.n, i, ql);
    const double nr = load_unit4(g4.quat_r, g4.n, i, qr);
    double R[4][4];
    {
        double L[4][4], Rr[4][4];
        rot_left(ql, L);
        rot_right(qr, Rr);
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c)
                R[r][c] = L[r][0] * Rr[0][c] + L[r][1] * Rr[1][c] + L[r][2] * Rr[2][c] + L[r][3] * Rr[3][c];
    }
    double S4[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = r; c < 4; ++c) {
            double acc = 0;
            for (int k = 0; k < 4; ++k) acc += R[r][k] * s[k] * s[k] * R[c][k];
            S4[r][c] = acc;
            S4[c][r] = acc;
        }
    const double c = S4[3][3], ic = 1.0 / c;
    const double b[3] = {S4[0][3], S4[1][3], S4[2][3]};
    const double mu0[3] = {(double)g4.mean[i], (double)g4.mean[n + i], (double)g4.mean[2 * n + i]};
    const double mt = (double)g4.mean_t[i];
    const double sig = sigmoid((double)g4.opacity[i]);
    double gmu[3] = {0, 0, 0}, gmt = 0, gsig = 0;
    double Ss[4][4];  // accumulated Sigma4-bar + Sigma4-bar^T
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) Ss[r][k] = 0.0;
    float gsh[48];
    for (int k = 0; k < 48; ++k) gsh[k] = 0.f;
    if constexpr (TIME)
        for (int k = 0; k < 48 * g4.sh_t_deg; ++k) gr.sh_t[(size_t)k * n + i] = 0.f;  // accumulated per view below
    double stat_g = 0.0;
    int stat_n = 0;
    for (int v = 0; v < n_views; ++v) {
        if (recs[(size_t)v * N + i].d.w == 0u) continue;  // covers no pixel in this view
        const ViewParams& V = views[v];
        const double delta = V.time - mt;
        const double pt = exp(-(delta * delta) * 0.5 * ic);
        WorldF w;
        for (int k = 0; k < 3; ++k) w.mu[k] = mu0[k] + b[k] * ic * delta;
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) w.S[r][k] = S4[r][k] - b[r] * b[k] * ic;
        w.op = sig * pt;
        if (st.grad || st.vis || st.step_vis) {
            const float* e = g2 + ((size_t)v * N + i) * kG2Stride;
            stat_g += ndc_grad_norm(e[0], e[1], kLn2 * w.op, V.W, V.H);
            ++stat_n;
        }
        ProjF p;
        project(V, w, p);
        double gmc[3], Sb[3][3], gop;
        if constexpr (TIME) {
            TimeColour tc;
            tc.g = &g4;
            tc.i = i;
            tc.gsht = gr.sh_t;
            time_weights(g4, i, V.time, tc.w, tc.dw);
            proj_bwd<true>(V, w, p, g4.sh, g4.n, i, g2 + ((size_t)v * N + i) * kG2Stride, 1, gmc, Sb, gop, gsh, &tc,
                           &gmt);
        } else {
            proj_bwd<false>(V, w, p, g4.sh, g4.n, i, g2 + ((size_t)v * N + i) * kG2Stride, 1, gmc, Sb, gop, gsh);
        }
        // effective opacity sigma * p(t); p(t) = exp(-delta^2 / (2 c))
        gsig += gop * pt;
        const double gpt = gop * sig;
        const double mub = gmc[0] * b[0] + gmc[1] * b[1] + gmc[2] * b[2];
        gmt += gpt * pt * delta * ic - mub * ic;
        double gc = gpt * pt * delta * delta * 0.5 * ic * ic - mub * delta * ic * ic;
        double bSb = 0.0;
        for (int r = 0; r < 3; ++r) {
            double row = 0.0;
            for (int k = 0; k < 3; ++k) row += Sb[r][k] * b[k];
            bSb += b[r] * row;
            // b-bar (mean and covariance terms); Sb is symmetric
            const double gb = gmc[r] * delta * ic - 2.0 * row * ic;
            Ss[r][3] += gb;
            Ss[3][r] += gb;
            gmu[r] += gmc[r];
        }
        gc += bSb * ic * ic;
        Ss[3][3] += 2.0 * gc;
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) Ss[r][k] += 2.0 * Sb[r][k];
    }
    // Sigma4 = Lm Lm^T, Lm = R diag(s): Lbar = Ss Lm, Rbar = Lbar diag(s), sbar_j = (R^T Lbar)_jj
    double Rb[4][4];
    for (int r = 0; r < 4; ++r)
        for (int j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) acc += Ss[r][k] * R[k][j];
            Rb[r][j] = acc * s[j] * s[j];  // = Lbar * s
        }
    for (int j = 0; j < 4; ++j) {
        double acc = 0.0;
        for (int r = 0; r < 4; ++r) acc += R[r][j] * Rb[r][j];
        gr.log_scale[j * n + i] = (float)acc;  // sbar_j s_j = sum_r R_rj Lbar_rj s_j
    }
    // R = L Rr: Lbar = Rbar Rr^T, Rrbar = L^T Rbar; each entry is +/- one quaternion component
    double gl[4], grr[4];
    {
        double Rr[4][4];
        rot_right(qr, Rr);
        double Lb[4][4];
        for (int r = 0; r < 4; ++r)
            for (int c2 = 0; c2 < 4; ++c2)
                Lb[r][c2] = Rb[r][0] * Rr[c2][0] + Rb[r][1] * Rr[c2][1] + Rb[r][2] * Rr[c2][2] + Rb[r][3] * Rr[c2][3];
        gl[0] = Lb[0][0] + Lb[1][1] + Lb[2][2] + Lb[3][3];
        gl[1] = -Lb[0][1] + Lb[1][0] - Lb[2][3] + Lb[3][2];
        gl[2] = -Lb[0][2] + Lb[1][3] + Lb[2][0] - Lb[3][1];
        gl[3] = -Lb[0][3] - Lb[1][2] + Lb[2][1] + Lb[3][0];
    }
    {
        double L[4][4];
        rot_left(ql, L);
        double Rrb[4][4];
        for (int r = 0; r < 4; ++r)
            for (int c2 = 0; c2 < 4; ++c2)
                Rrb[r][c2] = L[0][r] * Rb[0][c2] + L[1][r] * Rb[1][c2] + L[2][r] * Rb[2][c2] + L[3][r] * Rb[3][c2];
        grr[0] = Rrb[0][0] + Rrb[1][1] + Rrb[2][2] + Rrb[3][3];
        grr[1] = -Rrb[0][1] + Rrb[1][0] + Rrb[2][3] - Rrb[3][2];
        grr[2] = -Rrb[0][2] - Rrb[1][3] + Rrb[2][0] + Rrb[3][1];
        grr[3] = -Rrb[0][3] + Rrb[1][2] - Rrb[2][1] + Rrb[3][0];
    }
    unit_bwd(ql, nl, gl, gr.quat_l + i, n);
    unit_bwd(qr, nr, grr, gr.quat_r + i, n);
    for (int k = 0; k < 3; ++k) gr.mean[k * n + i] = (float)gmu[k];
    gr.mean_t[i] = (float)gmt;
    gr.opacity[i] = (float)(gsig * sig * (1.0 - sig));
    write_stats(st, i, stat_g, stat_n);
    for (int k = 0; k < 48; ++k) gr.sh[k * n + i] = gsh[k];
}

__device__ inline void bwd_3d(const G3Ptr& g3, int i, int gidx, const ViewParams* __restrict__ views, int n_views,
                              int N, const Rec* __restrict__ recs, const float* __restrict__ g2, const G3Grad& gr,
                              const SetStats& st, int static_rows) {
    const size_t n = (size_t)g3.n;
    WorldF w;
    Cov3 z;
    world3(g3, i, w, z);
    double gmu[3] = {0, 0, 0}, gsig = 0;
    double Ss[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    float gsh[48];
    for (int k = 0; k < 48; ++k) gsh[k] = 0.f;
    double stat_g = 0.0;
    int stat_n = 0;
    // the views of a static group share one camera and one record: their
    // screen-space gradients are summed (by the adjoint itself when
    // static_rows) and taken through the projection once
    for (int v = 0; v < n_views; ++v) {
        const ViewParams& V = views[v];
        if (V.static_view != v) continue;                  // summed into its group's leader below
        if (recs[(size_t)v * N + gidx].d.w == 0u) continue;  // covers no pixel in this camera
        // (a view alone, or the group's sum already in its record: that record
        // as it is; otherwise the members' records summed here)
        float e[kG2Slots];
        for (int k = 0; k < kG2Slots; ++k) e[k] = 0.f;
        const float* direct = nullptr;
        if (static_rows || V.static_next < 0) {
            direct = g2 + ((size_t)v * N + gidx) * kG2Stride;
            if (st.grad || st.vis || st.step_vis) {
                stat_g += ndc_grad_norm(direct[0], direct[1], kLn2 * w.op, V.W, V.H);
                ++stat_n;
            }
        }
        for (int u = direct ? -1 : v; u >= 0; u = views[u].static_next) {
            const float* g = g2 + ((size_t)u * N + gidx) * kG2Stride;
            if (st.grad || st.vis || st.step_vis) {
                stat_g += ndc_grad_norm(g[0], g[1], kLn2 * w.op, views[u].W, views[u].H);
                ++stat_n;
            }
            for (int k = 0; k < kG2Slots; ++k) e[k] += g[k];
        }
        ProjF p;
        project(V, w, p);
        double gmc[3], Sb[3][3], gop;
        proj_bwd<false>(V, w, p, g3.sh, g3.n, i, direct ? direct : e, 1, gmc, Sb, gop, gsh);
        gsig += gop;
        for (int r = 0; r < 3; ++r) {
            gmu[r] += gmc[r];
            for (int k = 0; k < 3; ++k) Ss[r][k] += 2.0 * Sb[r][k];
        }
    }
    double Rb[3][3];
    for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Ss[r][k] * z.R[k][j];
            Rb[r][j] = acc * z.s[j] * z.s[j];
        }
    for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r) acc += z.R[r][j] * Rb[r][j];
        gr.log_scale[j * n + i] = (float)acc;
    }
    const double qw = z.q[0], qx = z.q[1], qy = z.q[2], qz = z.q[3];
    double gq[4];
    gq[0] = 2.0 * (-qz * Rb[0][1] + qy * Rb[0][2] + qz * Rb[1][0] - qx * Rb[1][2] - qy * Rb[2][0] + qx * Rb[2][1]);
    gq[1] = 2.0 * (qy * Rb[0][1] + qz * Rb[0][2] + qy * Rb[1][0] - 2.0 * qx * Rb[1][1] - qw * Rb[1][2] +
                   qz * Rb[2][0] + qw * Rb[2][1] - 2.0 * qx * Rb[2][2]);
    gq[2] = 2.0 * (-2.0 * qy * Rb[0][0] + qx * Rb[0][1] + qw * Rb[0][2] + qx * Rb[1][0] + qz * Rb[1][2] -
                   qw * Rb[2][0] + qz * Rb[2][1] - 2.0 * qy * Rb[2][2]);
    gq[3] = 2.0 * (-2.0 * qz * Rb[0][0] - qw * Rb[0][1] + qx * Rb[0][2] + qw * Rb[1][0] - 2.0 * qz * Rb[1][1] +
                   qy * Rb[1][2] + qx * Rb[2][0] + qy * Rb[2][1]);
    unit_bwd(z.q, z.nq, gq, gr.quat + i, n);
    for (int k = 0; k < 3; ++k) gr.mean[k * n + i] = (float)gmu[k];
    gr.opacity[i] = (float)(gsig * z.sig * (1.0 - z.sig));
    write_stats(st, i, stat_g, stat_n);
    for (int k = 0; k < 48; ++k) gr.sh[k * n + i] = gsh[k];
}

// One launch for both sets: workgroups [0, nb4) take the 4D Gaussians (the
// longer threads, started first), the rest the 3D ones.  Both paths hold one
// wave per SIMD (FP64 state of 400+ registers), so sharing the launch costs no
// occupancy and lets the two sets fill the machine together.
// TIME: the 4D set carries time coefficients of its colour.
template <bool TIME>
__global__ void __launch_bounds__(128) k_preprocess_bwd(G3Ptr g3, G4Ptr g4, int nb4, const ViewParams* __restrict__ views,
                                                        int n_views, const Rec* __restrict__ recs,
                                                        const float* __restrict__ g2, G3Grad gr3, G4Grad gr4,
                                                        SetStats st3, SetStats st4, int static_rows,
                                                        Status* status) {
    const int N = g3.n + g4.n;
    if (blockIdx.x == 0 && threadIdx.x == 0) status->g2_dirty = 1ull;  // (read by the next backward's prologue)
    if ((int)blockIdx.x < nb4) {
        const int g = blockIdx.x * blockDim.x + threadIdx.x;
        if (g < g4.n) bwd_4d<TIME>(g4, g, views, n_views, N, recs, g2, gr4, st4);
    } else {
        const int i = (blockIdx.x - nb4) * blockDim.x + threadIdx.x;
        if (i < g3.n) bwd_3d(g3, i, g4.n + i, views, n_views, N, recs, g2, gr3, st3, static_rows);
    }
}

// ---------------------------------------------------------------------------
// Per-call view table: widened to FP64, camera centre -R^T t, tile bookkeeping.
// ---------------------------------------------------------------------------
__device__ void write_views(const ViewTableIn& in, ViewParams* out) {
    int tile_base = 0, super_base = 0;
    long long pix_base = 0;
    const int S = super_factor(in.tile);
    for (int v = 0; v < in.n; ++v) {
        const ViewIn& s = in.v[v];
        ViewParams p;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) p.R[3 * i + j] = (double)s.M[4 * i + j];
            p.T[i] = (double)s.M[4 * i + 3];
        }
        for (int j = 0; j < 3; ++j) p.campos[j] = -(p.R[j] * p.T[0] + p.R[3 + j] * p.T[1] + p.R[6 + j] * p.T[2]);
        p.fx = s.fx; p.fy = s.fy; p.cx = s.cx; p.cy = s.cy; p.time = s.t;
        for (int c = 0; c < 3; ++c) p.bg[c] = s.bg[c];
        p.W = s.W; p.H = s.H;
        p.tiles_x = ceil_div(s.W, in.tile);
        p.tiles_y = ceil_div(s.H, in.tile);
        p.tile_base = tile_base;
        p.pix_base = pix_base;
        p.sx = ceil_div(p.tiles_x, S);
        p.sy = ceil_div(p.tiles_y, S);
        p.super_base = super_base;
        p.static_view = in.share[v].static_view;
        p.static_group = in.share[v].static_group;
        p.static_super_base = in.share[v].static_super_base;
        p.static_next = in.share[v].static_next;
        p.group_leader = in.share[v].group_leader;
        p.pad = 0;
        super_base += p.sx * p.sy;
        tile_base += p.tiles_x * p.tiles_y;
        pix_base += (long long)s.W * s.H;
        out[v] = p;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
// Start of a forward call: the view table, cleared status and list-slot bases,
// and empty tile ranges, in one launch.
__global__ void __launch_bounds__(256) k_init_state(ViewTableIn in, ViewParams* views, Status* status,
                                                    unsigned long long* pair_base,
                                                    unsigned long long* ranges, size_t n_range_words) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) write_views(in, views);
        if (threadIdx.x < sizeof(Status) / 8) (&status->flags)[threadIdx.x] = 0ull;
        for (int v = threadIdx.x; v <= in.n; v += blockDim.x) pair_base[v] = 0ull;
    }
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_range_words;
         i += (size_t)gridDim.x * blockDim.x)
        ranges[i] = 0ull;
}

void launch_init_state(const ViewTableIn& in, ViewParams* views, Status* status, unsigned long long* pair_base,
                       unsigned long long* ranges, size_t n_range_words, hipStream_t st) {
    const int nb = (int)std::max<size_t>(1, std::min<size_t>(1024, (n_range_words + 255) / 256));
    k_init_state<<<nb, 256, 0, st>>>(in, views, status, pair_base, ranges, n_range_words);
}

void launch_preprocess(const G3Ptr& g3, const G4Ptr& g4, const ViewParams* views, int v0, int nv, int shared,
                       Rec* recs, uint32_t* dkeys, uint32_t* dvals, float* g2, hipStream_t st) {
    const int N = g3.n + g4.n;
    if (N == 0 || nv == 0) return;
    k_preprocess<<<dim3(ceil_div(N, 256), nv), 256, 0, st>>>(g3, g4, views, v0, shared, recs, dkeys, dvals, g2);
}

void launch_preprocess_bwd(const G3Ptr& g3, const G4Ptr& g4, const ViewParams* views, int n_views, const Rec* recs,
                           const float* g2, const G3Grad& gr3, const G4Grad& gr4, const SetStats& st3,
                           const SetStats& st4, int static_rows, Status* status, hipStream_t st) {
    const int N = g3.n + g4.n;
    const int nb4 = ceil_div(g4.n, 128), nb3 = ceil_div(g3.n, 128);
    const int nb = std::max(1, nb4 + nb3);  // (one workgroup at least: it marks the records used)
    if (g4.sh_t_deg > 0 && N > 0)
        k_preprocess_bwd<true><<<nb, 128, 0, st>>>(g3, g4, nb4, views, n_views, recs, g2, gr3, gr4, st3, st4,
                                                   static_rows, status);
    else
        k_preprocess_bwd<false><<<nb, 128, 0, st>>>(g3, g4, nb4, views, n_views, recs, g2, gr3, gr4, st3, st4,
                                                    static_rows, status);
}

}  // namespace h4d

namespace h4d {

// Screen-space splats given directly (Alg. 1 without the projection steps):
// the same record format, pixel square computed in FP64 from (u, v, r).
__global__ void __launch_bounds__(256) k_splats_to_records(int n, const float* __restrict__ u,
                                                           const float* __restrict__ v,
                                                           const float* __restrict__ conic,
                                                           const float* __restrict__ opacity,
                                                           const float* __restrict__ rgb,
                                                           const int32_t* __restrict__ radius,
                                                           const float* __restrict__ depth,
                                                           const uint8_t* __restrict__ visible, int W, int H,
                                                           Rec* __restrict__ recs, uint32_t* __restrict__ dkeys,
                                                           uint32_t* __restrict__ dvals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec rec;
    rec.a = make_float4(0.f, 0.f, 0.f, 0.f);
    rec.b = rec.a;
    rec.c = rec.a;
    rec.d = make_uint4(0u, 0u, 0u, 0u);
    uint32_t key = kCulledKey;
    const int r = radius[i];
    if (visible[i] && r >= 0) {
        const double uu = u[i], vv = v[i];
        const int x0 = max(0, (int)ceil(uu - r - 0.5)), x1 = min(W - 1, (int)floor(uu + r - 0.5));
        const int y0 = max(0, (int)ceil(vv - r - 0.5)), y1 = min(H - 1, (int)floor(vv + r - 0.5));
        if (x0 <= x1 && y0 <= y1) {
            const double s = -0.5 * 1.4426950408889634;
            const double fu = floor(uu), fv = floor(vv);
            rec.a = make_float4((float)(uu - fu), (float)(vv - fv), (float)((double)conic[i] * s),
                                (float)((double)conic[(size_t)n + i] * 2.0 * s));
            rec.b = make_float4((float)((double)conic[2 * (size_t)n + i] * s), opacity[i], rgb[i], rgb[(size_t)n + i]);
            rec.c = make_float4(rgb[2 * (size_t)n + i], (float)fu, (float)fv, depth[i]);
            rec.d = make_uint4((uint32_t)x0 | ((uint32_t)x1 << 16), (uint32_t)y0 | ((uint32_t)y1 << 16), (uint32_t)r, 1u);
            key = __float_as_uint(depth[i]);
        }
    }
    recs[i] = rec;
    dkeys[i] = key;
    dvals[i] = (uint32_t)i;
}

void launch_splats_to_records(int n, const float* u, const float* v, const float* conic, const float* opacity,
                              const float* rgb, const int32_t* radius, const float* depth, const uint8_t* visible,
                              int W, int H, Rec* recs, uint32_t* dkeys, uint32_t* dvals, hipStream_t st) {
    if (n == 0) return;
    k_splats_to_records<<<ceil_div(n, 256), 256, 0, st>>>(n, u, v, conic, opacity, rgb, radius, depth, visible, W, H,
                                                          recs, dkeys, dvals);
}

}  // namespace h4d

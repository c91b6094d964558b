/*
 * FP64 CPU oracle for the hybrid 3D/4D Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * definition that the HIP path is checked against.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (paper: "Hybrid 3D-4D Gaussian Splatting for Fast Dynamic
 * Scene Representation"):
 *   - activations and covariance  Sigma = R S S^T R^T              (Sec. 3.1, Eq. 2)
 *   - 4D rotation R = R_l(q_l) R_r(q_r)                            (Sec. 3.2, Eq. 4)
 *   - conditional mean / covariance of a 4D Gaussian at time t     (Sec. 3.2, Eq. 5-6)
 *   - temporal marginal opacity (inherited from 4DGS, referenced at the end of Sec. 3.2)
 *   - one merged list of 4D and 3D Gaussians, projected, keyed by (tile, depth),
 *     sorted and blended front to back                              (Sec. 4.3, Alg. 1, Eq. 3)
 *   - the exact adjoint of all of the above (the paper names an efficient backward
 *     pass, Sec. 5.2, without describing it; the adjoint is fixed by the forward)
 *   - static identification exp(s_t) > tau and 4D->3D conversion   (Sec. 4.1-4.2, Eq. 7-9)
 *   - an Adam step (the paper does not state its optimiser; textbook Kingma-Ba)
 *
 * Readings of what the paper leaves open (constants of the 3DGS lineage, camera
 * model, contribution region, depth key precision) are listed in the repository's
 * design notes; each is marked "reading" where it is used below.
 *
 * Everything is templated on the scalar type S: S = double for the oracle itself,
 * S = Dual for a forward-mode JVP used to pin the hand-written adjoint.
 * Arithmetic is FP64 throughout; compile without -ffast-math.
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py against
 * closed forms, brute force, invariants, finite differences or forward-mode AD.
 * Whole images have no printed worked example in the paper: beyond those pins,
 * image values are "parity unpinned".
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>
#include <omp.h>

namespace orc {

// ---------------------------------------------------------------------------
// Dual numbers (forward-mode derivative along one tangent direction).
// ---------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double x) : v(x), d(0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, a.d * e); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), a.d * std::cos(a.v)); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -a.d * std::sin(a.v)); }
inline Dual acos(Dual a) { return Dual(std::acos(a.v), -a.d / std::sqrt(1.0 - a.v * a.v)); }
inline Dual atan2(Dual y, Dual x) {
    double r2 = x.v * x.v + y.v * y.v;
    return Dual(std::atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2);
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::exp; using std::log; using std::sqrt; using std::sin; using std::cos; using std::acos; using std::atan2;

// ---------------------------------------------------------------------------
// Fixed constants of the rasterizer (reading: the 3DGS-lineage constants, since
// the paper builds on that implementation, Sec. 4.3, without restating them).
// ---------------------------------------------------------------------------
constexpr double kNear = 0.2;           // near-plane cull on camera-space z
constexpr double kMinAlpha = 1.0 / 255; // contributions below this are skipped
constexpr double kMaxAlpha = 0.99;      // alpha clamp
constexpr double kMinT = 1e-4;          // stop before transmittance would drop below this
constexpr double kDilate = 0.3;         // screen-space low-pass added to the 2D covariance
constexpr double kClampFov = 1.3;       // Jacobian clamp as a multiple of the half field of view
constexpr double kEigFloor = 0.1;       // floor of the eigenvalue discriminant
constexpr double kSigmas = 3.0;         // screen radius in standard deviations
constexpr double kShOffset = 0.5;       // SH colour offset (then clamped at 0)
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// ABI structs (mirrored by ctypes in oracle/__init__.py).
// ---------------------------------------------------------------------------
extern "C" {
struct OScene {
    int32_t n3;
    const float *mean3, *ls3, *q3, *op3, *sh3;              // [3][n3] [3][n3] [4][n3] [n3] [48][n3]
    int32_t n4;
    const float *mean4, *mt4, *ls4, *ql4, *qr4, *op4, *sh4; // [3] [1] [4] [4] [4] [1] [48] x n4
    int32_t sht_deg;     // time degree D of the 4D colour (0: plain SH)
    double sht_period;   // period T of its cosine terms
    const float *sht4;   // [48 D] x n4: coefficients of cos(2 pi n (t - mu_t) / T), n = 1 .. D
};
struct OTangent {  // same layout as OScene, float64, any pointer may be null (= zero tangent)
    const double *mean3, *ls3, *q3, *op3, *sh3;
    const double *mean4, *mt4, *ls4, *ql4, *qr4, *op4, *sh4;
    const double *sht4;
};
struct OGrad {     // float64 outputs, same layout as OScene (sht4 may be null when D = 0)
    double *mean3, *ls3, *q3, *op3, *sh3;
    double *mean4, *mt4, *ls4, *ql4, *qr4, *op4, *sh4;
    double *sht4;
};
struct OView {
    double R[9], T[3];   // world -> camera, row-major
    double fx, fy, cx, cy;
    int32_t W, H;
    double time;
    double bg[3];
};
}

// ---------------------------------------------------------------------------
// Parameters of one Gaussian of the merged list: index g < n4 is the 4D row g,
// g >= n4 is the 3D row g - n4 (Alg. 1 projects the 4D set first, then appends
// the 3D set to the same screen-space array M').
// ---------------------------------------------------------------------------
constexpr int kMaxTimeDeg = 2;
template <class S> struct Param {
    bool is4d;
    S mu[3], mt, ls[4], q[4], q2[4], op, sh[48];
    int sht_deg;       // time degree of the colour (4D only)
    double period;
    S sht[48 * kMaxTimeDeg];
};

template <class S> inline S mk(float x, const double* tan, size_t idx) {
    if constexpr (std::is_same<S, double>::value) { (void)tan; (void)idx; return (double)x; }
    else return S((double)x, tan ? tan[idx] : 0.0);
}

template <class S> void load_param(const OScene& sc, const OTangent* tg, int g, Param<S>& P) {
    const int n4 = sc.n4;
    if (g < n4) {
        const size_t n = (size_t)n4, i = (size_t)g;
        P.is4d = true;
        for (int k = 0; k < 3; ++k) P.mu[k] = mk<S>(sc.mean4[k * n + i], tg ? tg->mean4 : nullptr, k * n + i);
        P.mt = mk<S>(sc.mt4[i], tg ? tg->mt4 : nullptr, i);
        for (int k = 0; k < 4; ++k) P.ls[k] = mk<S>(sc.ls4[k * n + i], tg ? tg->ls4 : nullptr, k * n + i);
        for (int k = 0; k < 4; ++k) P.q[k] = mk<S>(sc.ql4[k * n + i], tg ? tg->ql4 : nullptr, k * n + i);
        for (int k = 0; k < 4; ++k) P.q2[k] = mk<S>(sc.qr4[k * n + i], tg ? tg->qr4 : nullptr, k * n + i);
        P.op = mk<S>(sc.op4[i], tg ? tg->op4 : nullptr, i);
        for (int k = 0; k < 48; ++k) P.sh[k] = mk<S>(sc.sh4[k * n + i], tg ? tg->sh4 : nullptr, k * n + i);
        P.sht_deg = sc.sht_deg;
        P.period = sc.sht_period;
        for (int k = 0; k < 48 * sc.sht_deg; ++k)
            P.sht[k] = mk<S>(sc.sht4[k * n + i], tg ? tg->sht4 : nullptr, k * n + i);
    } else {
        const size_t n = (size_t)sc.n3, i = (size_t)(g - n4);
        P.is4d = false;
        for (int k = 0; k < 3; ++k) P.mu[k] = mk<S>(sc.mean3[k * n + i], tg ? tg->mean3 : nullptr, k * n + i);
        P.mt = S(0.0);
        for (int k = 0; k < 3; ++k) P.ls[k] = mk<S>(sc.ls3[k * n + i], tg ? tg->ls3 : nullptr, k * n + i);
        P.ls[3] = S(0.0);
        for (int k = 0; k < 4; ++k) P.q[k] = mk<S>(sc.q3[k * n + i], tg ? tg->q3 : nullptr, k * n + i);
        for (int k = 0; k < 4; ++k) P.q2[k] = S(0.0);
        P.op = mk<S>(sc.op3[i], tg ? tg->op3 : nullptr, i);
        for (int k = 0; k < 48; ++k) P.sh[k] = mk<S>(sc.sh3[k * n + i], tg ? tg->sh3 : nullptr, k * n + i);
        P.sht_deg = 0;
        P.period = 1.0;
    }
}

// Colour coefficients of a Gaussian at time t (4D spherindrical harmonics, the
// colour model 4D Gaussian splatting uses): for a 4D Gaussian of time degree
// D, c_j = sh_j + sum_{n=1..D} cos(2 pi n (t - mu_t) / T) sht_{n,j}; otherwise
// c_j = sh_j.
template <class S> void sh_at(const Param<S>& P, double time, S c[48]) {
    for (int j = 0; j < 48; ++j) c[j] = P.sh[j];
    if (!P.is4d) return;
    for (int n = 1; n <= P.sht_deg; ++n) {
        const S w = cos(S(2.0 * M_PI * n / P.period) * (S(time) - P.mt));
        for (int j = 0; j < 48; ++j) c[j] += w * P.sht[(n - 1) * 48 + j];
    }
}

// ---------------------------------------------------------------------------
// Activations and rotations.
// ---------------------------------------------------------------------------
template <class S> inline S sigmoid(S x) { return S(1.0) / (S(1.0) + exp(-x)); }

template <class S> inline void normalize4(const S q[4], S out[4], S* norm = nullptr) {
    S n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) out[k] = q[k] / n;
    if (norm) *norm = n;
}

// Rotation matrix of a unit quaternion (w, x, y, z), Hamilton convention:
// R v = q v q^*.  Eq. 9's inverse map (R32 - R23 = 4wx, ...) fixes this convention.
template <class S> void quat_to_rot(const S q[4], S R[3][3]) {
    const S w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = S(1.0) - S(2.0) * (y * y + z * z); R[0][1] = S(2.0) * (x * y - w * z); R[0][2] = S(2.0) * (x * z + w * y);
    R[1][0] = S(2.0) * (x * y + w * z); R[1][1] = S(1.0) - S(2.0) * (x * x + z * z); R[1][2] = S(2.0) * (y * z - w * x);
    R[2][0] = S(2.0) * (x * z - w * y); R[2][1] = S(2.0) * (y * z + w * x); R[2][2] = S(1.0) - S(2.0) * (x * x + y * y);
}

// Eq. 4: the left matrix built from (a, b, c, d) and the right one from (p, q, r, s).
template <class S> void left_iso(const S q[4], S L[4][4]) {
    const S a = q[0], b = q[1], c = q[2], d = q[3];
    L[0][0] = a;  L[0][1] = -b; L[0][2] = -c; L[0][3] = -d;
    L[1][0] = b;  L[1][1] = a;  L[1][2] = -d; L[1][3] = c;
    L[2][0] = c;  L[2][1] = d;  L[2][2] = a;  L[2][3] = -b;
    L[3][0] = d;  L[3][1] = -c; L[3][2] = b;  L[3][3] = a;
}
template <class S> void right_iso(const S q[4], S Rr[4][4]) {
    const S p = q[0], qq = q[1], r = q[2], s = q[3];
    Rr[0][0] = p;  Rr[0][1] = -qq; Rr[0][2] = -r; Rr[0][3] = -s;
    Rr[1][0] = qq; Rr[1][1] = p;   Rr[1][2] = s;  Rr[1][3] = -r;
    Rr[2][0] = r;  Rr[2][1] = -s;  Rr[2][2] = p;  Rr[2][3] = qq;
    Rr[3][0] = s;  Rr[3][1] = r;   Rr[3][2] = -qq; Rr[3][3] = p;
}
template <class S, int N> void matmul(const S A[N][N], const S B[N][N], S C[N][N]) {
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            S acc = S(0.0);
            for (int k = 0; k < N; ++k) acc += A[i][k] * B[k][j];
            C[i][j] = acc;
        }
}
// Sigma = R diag(s^2) R^T  (Eq. 2; its 4D analogue for the 4D set - reading)
template <class S, int N> void cov_from(const S R[N][N], const S s[N], S Sg[N][N]) {
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            S acc = S(0.0);
            for (int k = 0; k < N; ++k) acc += R[i][k] * s[k] * s[k] * R[j][k];
            Sg[i][j] = acc;
        }
}

// ---------------------------------------------------------------------------
// World-space stage: covariance, slicing at time t (Eq. 5-6) and temporal opacity.
// ---------------------------------------------------------------------------
template <class S> struct Geo {
    S mu[3];       // mean at time t
    S Sg[3][3];    // covariance at time t
    S op;          // effective opacity sigma * p(t)
    S sig;         // sigmoid(opacity logit)
    S pt;          // temporal marginal p(t) (1 for 3D)
};

template <class S> void world(const Param<S>& P, double time, Geo<S>& G) {
    G.sig = sigmoid(P.op);
    if (P.is4d) {
        S s[4];
        for (int k = 0; k < 4; ++k) s[k] = exp(P.ls[k]);
        S ql[4], qr[4];
        normalize4(P.q, ql);
        normalize4(P.q2, qr);
        S L[4][4], Rr[4][4], R[4][4], Sg4[4][4];
        left_iso(ql, L);
        right_iso(qr, Rr);
        matmul<S, 4>(L, Rr, R);
        cov_from<S, 4>(R, s, Sg4);
        // Eq. 5-6 with index 4 = time: A = Sigma_{1:3,1:3}, b = Sigma_{1:3,4}, c = Sigma_{4,4}
        const S c = Sg4[3][3];
        const S delta = S(time) - P.mt;
        for (int i = 0; i < 3; ++i) G.mu[i] = P.mu[i] + Sg4[i][3] / c * delta;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) G.Sg[i][j] = Sg4[i][j] - Sg4[i][3] * Sg4[3][j] / c;
        // temporal marginal, unnormalised: exp(-delta^2 / (2 c)) (reading, 4DGS)
        G.pt = exp(-(delta * delta) / (S(2.0) * c));
    } else {
        S s[3];
        for (int k = 0; k < 3; ++k) s[k] = exp(P.ls[k]);
        S q[4], R[3][3];
        normalize4(P.q, q);
        quat_to_rot(q, R);
        cov_from<S, 3>(R, s, G.Sg);
        for (int i = 0; i < 3; ++i) G.mu[i] = P.mu[i];
        G.pt = S(1.0);
    }
    G.op = G.sig * G.pt;
}

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3, from the associated-Legendre
// definition (Condon-Shortley phase included in P_l^m), no constant table:
//   Y_l0 = K_l0 P_l^0(cos th),  Y_lm = sqrt2 K_lm P_l^m(cos th) cos(m ph),
//   Y_l,-m = sqrt2 K_lm P_l^m(cos th) sin(m ph),
//   K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  Index l*l + l + m.
// ---------------------------------------------------------------------------
inline double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

template <class S> void sh_basis(const S dir[3], S Y[16]) {
    const S z = dir[2];
    const S th = acos(z);
    const S st = sin(th);
    const S ph = atan2(dir[1], dir[0]);
    S P[4][4];  // P[l][m]
    for (int m = 0; m <= 3; ++m) {
        // P_m^m = (-1)^m (2m-1)!! sin^m
        double dfac = 1.0;
        for (int k = 1; k <= 2 * m - 1; k += 2) dfac *= k;
        S pmm = S((m % 2 ? -1.0 : 1.0) * dfac);
        for (int k = 0; k < m; ++k) pmm = pmm * st;
        P[m][m] = pmm;
        if (m + 1 <= 3) P[m + 1][m] = z * S(2.0 * m + 1) * pmm;
        for (int l = m + 2; l <= 3; ++l)
            P[l][m] = (S(2.0 * l - 1) * z * P[l - 1][m] - S(double(l + m - 1)) * P[l - 2][m]) / S(double(l - m));
    }
    for (int l = 0; l <= 3; ++l) {
        for (int m = 0; m <= l; ++m) {
            const double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fact(l - m) / fact(l + m));
            if (m == 0) {
                Y[l * l + l] = S(K) * P[l][0];
            } else {
                Y[l * l + l + m] = S(std::sqrt(2.0) * K) * P[l][m] * cos(S(double(m)) * ph);
                Y[l * l + l - m] = S(std::sqrt(2.0) * K) * P[l][m] * sin(S(double(m)) * ph);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Screen-space record of one Gaussian in one view (M' of Alg. 1).
// ---------------------------------------------------------------------------
template <class S> struct Rec {
    bool visible = false;   // survives every cull and covers >= 1 pixel
    bool culled = true;
    S u, v, depth;
    S Q[3];                 // conic (Q00, Q01, Q11) of the 2D covariance inverse
    S op;                   // effective opacity
    S rgb[3];
    int r = 0;              // integer screen radius
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;  // pixel square, inclusive
    float key = 0.f;        // FP32 depth key used for ordering (reading: kernel precision)
    int kinks = 0;          // which clamps are active: bit c = colour channel c at 0, bit 3/4 = x/y Jacobian
    double margin = 1.0;    // min relative margin of this Gaussian's FP64 discrete decisions
    bool key_shaky = false; // depth lies within kGlobalTol of a float32 rounding boundary
};

// An FP64 evaluation with a different operation order differs from this one by
// far less than this relative amount; decisions closer than that are flagged.
constexpr double kGlobalTol = 1e-11;

inline double frac_dist(double x) { return std::fabs(x - std::nearbyint(x)); }

// relative distance of x (> 0) to the nearest rounding boundary of float32
inline double f32_round_margin(double x) {
    float f = (float)x;
    double lo = std::nextafter(f, -INFINITY), hi = std::nextafter(f, INFINITY);
    double mlo = 0.5 * ((double)f + lo), mhi = 0.5 * ((double)f + hi);
    return std::min(std::fabs(x - mlo), std::fabs(x - mhi)) / std::fabs(x);
}

template <class S> void project(const OView& V, const Param<S>& P, const Geo<S>& G, Rec<S>& r) {
    r = Rec<S>();
    S pc[3];
    for (int i = 0; i < 3; ++i) pc[i] = S(V.R[3 * i]) * G.mu[0] + S(V.R[3 * i + 1]) * G.mu[1] + S(V.R[3 * i + 2]) * G.mu[2] + S(V.T[i]);
    double margin = std::min(std::fabs(val(pc[2]) - kNear) / kNear, std::fabs(val(G.op) - kMinAlpha) / kMinAlpha);
    r.margin = margin;
    // K1 (Alg. 1 CullGaussian; reading): near plane and effective opacity.  A
    // Gaussian culled by a hair keeps its square (still culled) so that the pixels
    // it could touch get flagged.
    const bool cull = val(pc[2]) <= kNear || val(G.op) < kMinAlpha;
    if (cull && (margin >= kGlobalTol || val(pc[2]) <= 0.5 * kNear)) return;
    const S z = pc[2];
    const S x = pc[0] / z, y = pc[1] / z;
    const double limx = kClampFov * (0.5 * V.W / V.fx), limy = kClampFov * (0.5 * V.H / V.fy);
    const S xt = val(x) > limx ? S(limx) : (val(x) < -limx ? S(-limx) : x);
    const S yt = val(y) > limy ? S(limy) : (val(y) < -limy ? S(-limy) : y);
    const int jkinks = (std::fabs(val(x)) > limx ? 8 : 0) | (std::fabs(val(y)) > limy ? 16 : 0);
    // EWA: J = d(pixel)/d(camera point) with the clamped ratios
    S J[2][3] = {{S(V.fx) / z, S(0.0), -S(V.fx) * xt / z}, {S(0.0), S(V.fy) / z, -S(V.fy) * yt / z}};
    S M[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = J[i][0] * S(V.R[j]) + J[i][1] * S(V.R[3 + j]) + J[i][2] * S(V.R[6 + j]);
    S S2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            S acc = S(0.0);
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += M[i][k] * G.Sg[k][l] * M[j][l];
            S2[i][j] = acc;
        }
    const S a = S2[0][0] + S(kDilate), b = S2[0][1], d = S2[1][1] + S(kDilate);
    const S det = a * d - b * b;
    margin = std::min(margin, std::fabs(val(det)) / (val(a) * val(d)));
    r.margin = margin;
    if (val(det) <= 0.0) return;
    r.Q[0] = d / det; r.Q[1] = -b / det; r.Q[2] = a / det;
    const S mid = S(0.5) * (a + d);
    const double disc = std::max(kEigFloor, val(mid) * val(mid) - val(det));
    const double lam = val(mid) + std::sqrt(disc);
    const double rr = kSigmas * std::sqrt(lam);
    margin = std::min(margin, frac_dist(rr) / rr);
    r.r = (int)std::ceil(rr);
    r.u = S(V.fx) * x + S(V.cx);
    r.v = S(V.fy) * y + S(V.cy);
    // pixel (i, j) is sampled at (i + 0.5, j + 0.5); it lies in the square iff
    // |i + 0.5 - u| <= r and |j + 0.5 - v| <= r  (reading: contribution region)
    const double ulo = val(r.u) - r.r - 0.5, uhi = val(r.u) + r.r - 0.5;
    const double vlo = val(r.v) - r.r - 0.5, vhi = val(r.v) + r.r - 0.5;
    for (double e : {ulo, uhi, vlo, vhi}) margin = std::min(margin, frac_dist(e) / std::max(1.0, std::fabs(e)));
    r.x0 = std::max(0, (int)std::ceil(ulo));
    r.x1 = std::min(V.W - 1, (int)std::floor(uhi));
    r.y0 = std::max(0, (int)std::ceil(vlo));
    r.y1 = std::min(V.H - 1, (int)std::floor(vhi));
    r.depth = z;
    r.key = (float)val(z);
    r.key_shaky = f32_round_margin(val(z)) < kGlobalTol;
    r.op = G.op;
    // colour: SH of the viewing direction from the camera centre
    const double C[3] = {-(V.R[0] * V.T[0] + V.R[3] * V.T[1] + V.R[6] * V.T[2]),
                         -(V.R[1] * V.T[0] + V.R[4] * V.T[1] + V.R[7] * V.T[2]),
                         -(V.R[2] * V.T[0] + V.R[5] * V.T[1] + V.R[8] * V.T[2])};
    S e[3] = {G.mu[0] - S(C[0]), G.mu[1] - S(C[1]), G.mu[2] - S(C[2])};
    const S en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    S dir[3] = {e[0] / en, e[1] / en, e[2] / en};
    S Y[16], cf[48];
    sh_basis(dir, Y);
    sh_at(P, V.time, cf);
    for (int ch = 0; ch < 3; ++ch) {
        S acc = S(kShOffset);
        for (int k = 0; k < 16; ++k) acc += cf[k * 3 + ch] * Y[k];
        r.rgb[ch] = val(acc) > 0.0 ? acc : S(0.0);
        if (!(val(acc) > 0.0)) r.kinks |= 1 << ch;
    }
    r.kinks |= jkinks;
    r.margin = margin;
    r.culled = cull;
    r.visible = !cull && (r.x0 <= r.x1) && (r.y0 <= r.y1);
}

// ---------------------------------------------------------------------------
// Alg. 1 CreateTiles / DuplicateWithKeys / SortByKeys / IdentifyTileRanges.
// The (tile, depth key, id) order is a total order; a per-tile std::sort of the
// bucket gives exactly the globally sorted pair list's per-tile ranges.
// ---------------------------------------------------------------------------
struct TileLists {
    int tx = 0, ty = 0, B = 16;
    std::vector<int64_t> start;  // [tiles + 1]
    std::vector<int32_t> ids;    // concatenated per-tile lists
};

// rect_grow: widen each square by this many pixels before binning (0 for the
// exact lists; 1 when the oracle wants to look at every pixel next to a square).
template <class GetRect>
void build_tiles(int n, int W, int H, int B, GetRect get, TileLists& tl) {
    tl.B = B;
    tl.tx = (W + B - 1) / B;
    tl.ty = (H + B - 1) / B;
    const int T = tl.tx * tl.ty;
    std::vector<int64_t> cnt(T + 1, 0);
    for (int g = 0; g < n; ++g) {
        int x0, x1, y0, y1; float key;
        if (!get(g, x0, x1, y0, y1, key)) continue;
        for (int ty = y0 / B; ty <= y1 / B; ++ty)
            for (int tx = x0 / B; tx <= x1 / B; ++tx) cnt[ty * tl.tx + tx]++;
    }
    tl.start.assign(T + 1, 0);
    for (int t = 0; t < T; ++t) tl.start[t + 1] = tl.start[t] + cnt[t];
    tl.ids.assign((size_t)tl.start[T], 0);
    std::vector<int64_t> fill(tl.start.begin(), tl.start.end() - 1);
    std::vector<float> keys((size_t)n, 0.f);
    for (int g = 0; g < n; ++g) {
        int x0, x1, y0, y1; float key;
        if (!get(g, x0, x1, y0, y1, key)) continue;
        keys[g] = key;
        for (int ty = y0 / B; ty <= y1 / B; ++ty)
            for (int tx = x0 / B; tx <= x1 / B; ++tx) tl.ids[fill[ty * tl.tx + tx]++] = g;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < T; ++t) {
        std::sort(tl.ids.begin() + tl.start[t], tl.ids.begin() + tl.start[t + 1], [&](int a, int b) {
            if (keys[a] != keys[b]) return keys[a] < keys[b];
            return a < b;
        });
    }
}

// ---------------------------------------------------------------------------
// Front-to-back blending of one pixel (Eq. 3; Alg. 1 BlendInOrder), with the
// discrete-decision margins used to flag pixels whose FP32 evaluation could
// legitimately take a different branch.
// ---------------------------------------------------------------------------
struct Blended {  // one blended entry, kept for the adjoint
    int g;
    double alpha, T, G, dx, dy;
    bool clamped;
};

constexpr double kEps32 = 5.9604644775390625e-08;  // 2^-24

template <class S, class Recs = std::vector<Rec<S>>>
void blend_pixel(int i, int j, const int32_t* list, int64_t len, const Recs& recs, const OView& V,
                 S C[3], S& Tout, int& nblend, bool& amb, std::vector<Blended>* keep) {
    const double x = i + 0.5, y = j + 0.5;
    S T = S(1.0);
    C[0] = C[1] = C[2] = S(0.0);
    nblend = 0;
    amb = false;
    double eT = 0.0;  // accumulated relative error bound of T for an FP32 evaluation
    int prev = -1;    // previous in-square candidate (for the depth-key tie check)
    for (int64_t k = 0; k < len; ++k) {
        const int g = list[k];
        const Rec<S>& r = recs[g];
        if (r.culled) continue;
        if (i < r.x0 || i > r.x1 || j < r.y0 || j > r.y1) continue;
        if (prev >= 0) {
            const Rec<S>& q = recs[prev];
            if ((r.key_shaky || q.key_shaky) && std::nextafter(q.key, INFINITY) >= r.key) amb = true;
        }
        prev = g;
        const S dx = S(x) - r.u, dy = S(y) - r.v;
        const S power = S(-0.5) * (r.Q[0] * dx * dx + S(2.0) * r.Q[1] * dx * dy + r.Q[2] * dy * dy);
        // Error bound of an FP32 evaluation of power and alpha (guard band), with
        // u = 2^-24: float32 conic and centre fraction (u each), at most three
        // roundings per term of the quadratic form, the offsets' rounding
        // u (1 + |d|), exp2 within 2 ulp, two more roundings for op * G.
        const double qa = val(r.Q[0]), qb = val(r.Q[1]), qc = val(r.Q[2]), ddx = val(dx), ddy = val(dy);
        const double terms = 0.5 * (std::fabs(qa) * ddx * ddx + 2 * std::fabs(qb * ddx * ddy) + std::fabs(qc) * ddy * ddy);
        const double epow = 4 * kEps32 * terms + std::fabs(qa * ddx + qb * ddy) * kEps32 * (1.0 + std::fabs(ddx)) +
                            std::fabs(qb * ddx + qc * ddy) * kEps32 * (1.0 + std::fabs(ddy)) +
                            kEps32 * std::fabs(val(power));
        const double ealpha = epow + 4 * kEps32;
        if (val(power) > 0.0) {
            if (val(r.op) >= kMinAlpha && 2 * epow > val(power)) amb = true;
            continue;
        }
        const S Gk = exp(power);
        const S ap = r.op * Gk;
        if (std::fabs(std::log(val(ap) / kMinAlpha)) < 2 * ealpha + 1e-7) amb = true;
        const bool clamped = val(ap) > kMaxAlpha;
        const S alpha = clamped ? S(kMaxAlpha) : ap;
        if (val(alpha) < kMinAlpha) continue;
        const S Tn = T * (S(1.0) - alpha);
        const double eTn = eT + (clamped ? 0.0 : val(alpha) * ealpha / (1.0 - val(alpha))) + 2 * kEps32;
        if (std::fabs(std::log(val(Tn) / kMinT)) < 2 * eTn + 1e-7) amb = true;
        if (val(Tn) < kMinT) break;  // this Gaussian is not blended
        for (int c = 0; c < 3; ++c) C[c] += r.rgb[c] * alpha * T;
        if (keep) keep->push_back(Blended{g, val(alpha), val(T), val(Gk), val(dx), val(dy), clamped});
        T = Tn;
        eT = eTn;
        ++nblend;
    }
    Tout = T;
}

// ---------------------------------------------------------------------------
// Whole-view forward: preprocess every Gaussian, bin, sort, blend.
// ---------------------------------------------------------------------------
template <class S>
void preprocess_all(const OScene& sc, const OTangent* tg, const OView& V, std::vector<Rec<S>>& recs) {
    const int N = sc.n3 + sc.n4;
    recs.assign(N, Rec<S>());
#pragma omp parallel for schedule(static)
    for (int g = 0; g < N; ++g) {
        Param<S> P;
        load_param(sc, tg, g, P);
        Geo<S> G;
        world(P, V.time, G);
        project(V, P, G, recs[g]);
    }
}

template <class S>
void render_view(const OScene& sc, const OTangent* tg, const OView& V, int B, S* img, S* Tfin, int32_t* nbl,
                 uint8_t* amb, std::vector<Rec<S>>* recs_out = nullptr) {
    std::vector<Rec<S>> recs;
    preprocess_all(sc, tg, V, recs);
    const int N = (int)recs.size();
    // lists widened by one pixel so that Gaussians whose decisions are marginal can
    // flag the pixels next to their square; the exact square test runs per pixel.
    TileLists tl;
    build_tiles(N, V.W, V.H, B,
                [&](int g, int& x0, int& x1, int& y0, int& y1, float& key) {
                    const Rec<S>& r = recs[g];
                    if (r.culled) return false;
                    x0 = std::max(0, r.x0 - 1); x1 = std::min(V.W - 1, r.x1 + 1);
                    y0 = std::max(0, r.y0 - 1); y1 = std::min(V.H - 1, r.y1 + 1);
                    key = r.key;
                    return x0 <= x1 && y0 <= y1;
                },
                tl);
    const int HW = V.W * V.H;
    std::vector<uint8_t> flag((size_t)HW, 0);
    // Gaussians with a marginal global decision flag every pixel of their widened square
    for (int g = 0; g < N; ++g) {
        const Rec<S>& r = recs[g];
        if (r.margin >= kGlobalTol || r.r == 0) continue;
        const int xa = std::max(0, r.x0 - 1), xb = std::min(V.W - 1, r.x1 + 1);
        const int ya = std::max(0, r.y0 - 1), yb = std::min(V.H - 1, r.y1 + 1);
        for (int j = ya; j <= yb; ++j)
            for (int i = xa; i <= xb; ++i) flag[(size_t)j * V.W + i] = 1;
    }
    const int T = tl.tx * tl.ty;
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < T; ++t) {
        const int tx = t % tl.tx, ty = t / tl.tx;
        const int32_t* list = tl.ids.data() + tl.start[t];
        const int64_t len = tl.start[t + 1] - tl.start[t];
        for (int j = ty * B; j < std::min(V.H, (ty + 1) * B); ++j)
            for (int i = tx * B; i < std::min(V.W, (tx + 1) * B); ++i) {
                S C[3], Tp;
                int nb;
                bool a;
                blend_pixel(i, j, list, len, recs, V, C, Tp, nb, a, nullptr);
                const size_t p = (size_t)j * V.W + i;
                for (int c = 0; c < 3; ++c) img[(size_t)c * HW + p] = C[c] + Tp * S(V.bg[c]);
                if (Tfin) Tfin[p] = Tp;
                if (nbl) nbl[p] = nb;
                if (amb) amb[p] = (uint8_t)(a || flag[p]);
            }
    }
    if (recs_out) recs_out->swap(recs);
}

// ---------------------------------------------------------------------------
// Adjoint (hand-written).  dL/dC per pixel -> per-Gaussian screen-space
// gradients -> per-parameter gradients.
// ---------------------------------------------------------------------------
struct G2 { double u, v, Q[3], op, rgb[3]; };

// derivative of the SH basis w.r.t. the direction, by three forward-mode passes
inline void sh_basis_grad(const double dir[3], double dY[16][3]) {
    for (int a = 0; a < 3; ++a) {
        Dual d[3] = {Dual(dir[0], a == 0), Dual(dir[1], a == 1), Dual(dir[2], a == 2)};
        Dual Y[16];
        sh_basis(d, Y);
        for (int k = 0; k < 16; ++k) dY[k][a] = Y[k].d;
    }
}

// per-Gaussian chain rule for one view; accumulates into grad arrays of Gaussian g
// gsh receives the gradient of this view's colour coefficients (sh_at);
// gsht (may be null) the accumulated gradient of the time coefficients.
void gaussian_bwd(const OScene& sc, int g, const OView& V, const G2& gs, double* gmu, double* gmt, double* gls,
                  double* gq, double* gq2, double* gop, double* gsh, double* gsht) {
    Param<double> P;
    load_param<double>(sc, nullptr, g, P);
    // ---- forward recomputation
    double s[4] = {0, 0, 0, 0};
    const int ns = P.is4d ? 4 : 3;
    for (int k = 0; k < ns; ++k) s[k] = std::exp(P.ls[k]);
    const double sig = 1.0 / (1.0 + std::exp(-P.op));
    double ql[4], qr[4], nl = 0, nr = 0;
    normalize4(P.q, ql, &nl);
    double L4[4][4], R4r[4][4], R4[4][4], Sg4[4][4], R3[3][3];
    double mu[3], Sg[3][3], pt = 1.0, delta = 0, c = 1;
    double bvec[3] = {0, 0, 0};
    if (P.is4d) {
        normalize4(P.q2, qr, &nr);
        left_iso(ql, L4);
        right_iso(qr, R4r);
        matmul<double, 4>(L4, R4r, R4);
        cov_from<double, 4>(R4, s, Sg4);
        c = Sg4[3][3];
        delta = V.time - P.mt;
        for (int i = 0; i < 3; ++i) bvec[i] = Sg4[i][3];
        for (int i = 0; i < 3; ++i) mu[i] = P.mu[i] + bvec[i] / c * delta;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Sg[i][j] = Sg4[i][j] - bvec[i] * bvec[j] / c;
        pt = std::exp(-delta * delta / (2 * c));
    } else {
        quat_to_rot(ql, R3);
        cov_from<double, 3>(R3, s, Sg);
        for (int i = 0; i < 3; ++i) mu[i] = P.mu[i];
    }
    const double* Rw = V.R;
    double pc[3];
    for (int i = 0; i < 3; ++i) pc[i] = Rw[3 * i] * mu[0] + Rw[3 * i + 1] * mu[1] + Rw[3 * i + 2] * mu[2] + V.T[i];
    const double z = pc[2], x = pc[0] / z, y = pc[1] / z;
    const double limx = kClampFov * (0.5 * V.W / V.fx), limy = kClampFov * (0.5 * V.H / V.fy);
    const bool cx_ = (x > limx) || (x < -limx), cy_ = (y > limy) || (y < -limy);
    const double xt = x > limx ? limx : (x < -limx ? -limx : x);
    const double yt = y > limy ? limy : (y < -limy ? -limy : y);
    double J[2][3] = {{V.fx / z, 0, -V.fx * xt / z}, {0, V.fy / z, -V.fy * yt / z}};
    double M[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = J[i][0] * Rw[j] + J[i][1] * Rw[3 + j] + J[i][2] * Rw[6 + j];
    double S2[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += M[i][k] * Sg[k][l] * M[j][l];
            S2[i][j] = acc;
        }
    const double a = S2[0][0] + kDilate, b = S2[0][1], d = S2[1][1] + kDilate;
    const double det = a * d - b * b;
    const double Q[2][2] = {{d / det, -b / det}, {-b / det, a / det}};
    const double Cc[3] = {-(Rw[0] * V.T[0] + Rw[3] * V.T[1] + Rw[6] * V.T[2]),
                          -(Rw[1] * V.T[0] + Rw[4] * V.T[1] + Rw[7] * V.T[2]),
                          -(Rw[2] * V.T[0] + Rw[5] * V.T[1] + Rw[8] * V.T[2])};
    double e[3] = {mu[0] - Cc[0], mu[1] - Cc[1], mu[2] - Cc[2]};
    const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    double dir[3] = {e[0] / en, e[1] / en, e[2] / en};
    double Y[16];
    sh_basis(dir, Y);

    // ---- colour adjoint (clamp at zero passes the gradient only where raw > 0)
    double gmu_c[3] = {0, 0, 0};
    double gdir[3] = {0, 0, 0};
    double dY[16][3], cf[48], gcf[48];
    sh_basis_grad(dir, dY);
    sh_at(P, V.time, cf);
    for (int j = 0; j < 48; ++j) gcf[j] = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        double raw = kShOffset;
        for (int k = 0; k < 16; ++k) raw += cf[k * 3 + ch] * Y[k];
        const double gc = raw > 0.0 ? gs.rgb[ch] : 0.0;
        if (gc == 0.0) continue;
        for (int k = 0; k < 16; ++k) {
            gcf[k * 3 + ch] += gc * Y[k];
            for (int a3 = 0; a3 < 3; ++a3) gdir[a3] += gc * cf[k * 3 + ch] * dY[k][a3];
        }
    }
    for (int j = 0; j < 48; ++j) gsh[j] += gcf[j];
    // time coefficients: dc_j/dsht_{n,j} = cos(phase_n); dc_j/dmu_t =
    // sum_n (2 pi n / T) sin(phase_n) sht_{n,j}, phase_n = 2 pi n (t - mu_t) / T
    if (P.is4d)
        for (int n = 1; n <= P.sht_deg; ++n) {
            const double k2 = 2.0 * M_PI * n / P.period, ph = k2 * (V.time - P.mt);
            double acc = 0.0;
            for (int j = 0; j < 48; ++j) {
                if (gsht) gsht[(n - 1) * 48 + j] += std::cos(ph) * gcf[j];
                acc += gcf[j] * P.sht[(n - 1) * 48 + j];
            }
            *gmt += k2 * std::sin(ph) * acc;
        }
    {
        const double dd = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
        for (int i = 0; i < 3; ++i) gmu_c[i] += (gdir[i] - dir[i] * dd) / en;
    }
    // ---- conic -> 2D covariance: Sbar = -Q Gbar Q with Gbar = [[Qa, Qb/2], [Qb/2, Qc]]
    const double Gb[2][2] = {{gs.Q[0], 0.5 * gs.Q[1]}, {0.5 * gs.Q[1], gs.Q[2]}};
    double S2b[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += Q[i][k] * Gb[k][l] * Q[l][j];
            S2b[i][j] = -acc;
        }
    // ---- 2D covariance = M Sigma M^T (+ dilation)
    double Sgb[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += M[k][i] * S2b[k][l] * M[l][j];
            Sgb[i][j] = acc;
        }
    double Mb[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 3; ++l) acc += S2b[i][k] * M[k][l] * Sg[l][j];
            Mb[i][j] = 2.0 * acc;
        }
    double Jb[2][3];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) Jb[i][j] = Mb[i][0] * Rw[3 * j] + Mb[i][1] * Rw[3 * j + 1] + Mb[i][2] * Rw[3 * j + 2];
    // ---- Jacobian entries -> camera point
    double pb[3] = {0, 0, 0};
    double xb = 0, yb = 0;
    pb[2] += Jb[0][0] * (-V.fx / (z * z)) + Jb[0][2] * (V.fx * xt / (z * z)) + Jb[1][1] * (-V.fy / (z * z)) +
             Jb[1][2] * (V.fy * yt / (z * z));
    const double xtb = Jb[0][2] * (-V.fx / z), ytb = Jb[1][2] * (-V.fy / z);
    if (!cx_) xb += xtb;
    if (!cy_) yb += ytb;
    xb += gs.u * V.fx;
    yb += gs.v * V.fy;
    pb[0] += xb / z;
    pb[1] += yb / z;
    pb[2] += -xb * pc[0] / (z * z) - yb * pc[1] / (z * z);
    for (int i = 0; i < 3; ++i) gmu_c[i] += Rw[i] * pb[0] + Rw[3 + i] * pb[1] + Rw[6 + i] * pb[2];
    // ---- effective opacity
    const double gsig = gs.op * pt;
    const double gpt = gs.op * sig;
    *gop += gsig * sig * (1.0 - sig);
    // ---- world stage
    if (P.is4d) {
        double gmt_ = gpt * pt * delta / c;
        double gc = gpt * pt * delta * delta / (2 * c * c);
        double gbv[3];
        double mub = gmu_c[0] * bvec[0] + gmu_c[1] * bvec[1] + gmu_c[2] * bvec[2];
        for (int i = 0; i < 3; ++i) {
            gmu[i] += gmu_c[i];
            gbv[i] = gmu_c[i] * delta / c;
        }
        gmt_ += -mub / c;
        gc += -mub * delta / (c * c);
        double bSb = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) bSb += bvec[i] * Sgb[i][j] * bvec[j];
        for (int i = 0; i < 3; ++i) {
            double acc = 0;
            for (int j = 0; j < 3; ++j) acc += (Sgb[i][j] + Sgb[j][i]) * bvec[j];
            gbv[i] += -acc / c;
        }
        gc += bSb / (c * c);
        *gmt += gmt_;
        double S4b[4][4] = {{0}};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S4b[i][j] = Sgb[i][j];
        for (int i = 0; i < 3; ++i) S4b[i][3] = gbv[i];
        S4b[3][3] = gc;
        // Sigma4 = Lm Lm^T with Lm = R4 diag(s): Lbar = (Sbar + Sbar^T) Lm
        double Lm[4][4], Lb[4][4], Rb[4][4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) Lm[i][j] = R4[i][j] * s[j];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double acc = 0;
                for (int k = 0; k < 4; ++k) acc += (S4b[i][k] + S4b[k][i]) * Lm[k][j];
                Lb[i][j] = acc;
            }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) Rb[i][j] = Lb[i][j] * s[j];
        for (int k = 0; k < 4; ++k) {
            double acc = 0;
            for (int i = 0; i < 4; ++i) acc += R4[i][k] * Lb[i][k];
            gls[k] += acc * s[k];
        }
        // R4 = L R_r: Lbar_l = R4bar R_r^T, Rbar_r = L^T R4bar
        double Lbl[4][4], Rbr[4][4];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double a1 = 0, a2 = 0;
                for (int k = 0; k < 4; ++k) {
                    a1 += Rb[i][k] * R4r[j][k];
                    a2 += L4[k][i] * Rb[k][j];
                }
                Lbl[i][j] = a1;
                Rbr[i][j] = a2;
            }
        // each matrix entry is +/- one quaternion component (Eq. 4 pattern)
        double gqlh[4], gqrh[4];
        gqlh[0] = Lbl[0][0] + Lbl[1][1] + Lbl[2][2] + Lbl[3][3];
        gqlh[1] = -Lbl[0][1] + Lbl[1][0] - Lbl[2][3] + Lbl[3][2];
        gqlh[2] = -Lbl[0][2] + Lbl[1][3] + Lbl[2][0] - Lbl[3][1];
        gqlh[3] = -Lbl[0][3] - Lbl[1][2] + Lbl[2][1] + Lbl[3][0];
        gqrh[0] = Rbr[0][0] + Rbr[1][1] + Rbr[2][2] + Rbr[3][3];
        gqrh[1] = -Rbr[0][1] + Rbr[1][0] + Rbr[2][3] - Rbr[3][2];
        gqrh[2] = -Rbr[0][2] - Rbr[1][3] + Rbr[2][0] + Rbr[3][1];
        gqrh[3] = -Rbr[0][3] + Rbr[1][2] - Rbr[2][1] + Rbr[3][0];
        double dl = 0, dr = 0;
        for (int k = 0; k < 4; ++k) { dl += ql[k] * gqlh[k]; dr += qr[k] * gqrh[k]; }
        for (int k = 0; k < 4; ++k) {
            gq[k] += (gqlh[k] - ql[k] * dl) / nl;
            gq2[k] += (gqrh[k] - qr[k] * dr) / nr;
        }
    } else {
        for (int i = 0; i < 3; ++i) gmu[i] += gmu_c[i];
        double Lm[3][3], Lb[3][3], Rb[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Lm[i][j] = R3[i][j] * s[j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += (Sgb[i][k] + Sgb[k][i]) * Lm[k][j];
                Lb[i][j] = acc;
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Rb[i][j] = Lb[i][j] * s[j];
        for (int k = 0; k < 3; ++k) {
            double acc = 0;
            for (int i = 0; i < 3; ++i) acc += R3[i][k] * Lb[i][k];
            gls[k] += acc * s[k];
        }
        const double w = ql[0], qx = ql[1], qy = ql[2], qz = ql[3];
        double gqh[4];
        gqh[0] = 2 * (-qz * Rb[0][1] + qy * Rb[0][2] + qz * Rb[1][0] - qx * Rb[1][2] - qy * Rb[2][0] + qx * Rb[2][1]);
        gqh[1] = 2 * (qy * Rb[0][1] + qz * Rb[0][2] + qy * Rb[1][0] - 2 * qx * Rb[1][1] - w * Rb[1][2] + qz * Rb[2][0] +
                      w * Rb[2][1] - 2 * qx * Rb[2][2]);
        gqh[2] = 2 * (-2 * qy * Rb[0][0] + qx * Rb[0][1] + w * Rb[0][2] + qx * Rb[1][0] + qz * Rb[1][2] - w * Rb[2][0] +
                      qz * Rb[2][1] - 2 * qy * Rb[2][2]);
        gqh[3] = 2 * (-2 * qz * Rb[0][0] - w * Rb[0][1] + qx * Rb[0][2] + w * Rb[1][0] - 2 * qz * Rb[1][1] + qy * Rb[1][2] +
                      qx * Rb[2][0] + qy * Rb[2][1]);
        double dq = 0;
        for (int k = 0; k < 4; ++k) dq += ql[k] * gqh[k];
        for (int k = 0; k < 4; ++k) gq[k] += (gqh[k] - ql[k] * dq) / nl;
    }
}

// Composite adjoint of one pixel (upstream gbar = dL/dC, 3 channels).
// acc(g) returns the accumulator of Gaussian g, or null to drop its terms.
template <class Recs, class Acc>
inline void blend_pixel_bwd(const std::vector<Blended>& bl, const Recs& recs, const double Tfin,
                            const double bg[3], const double gbar[3], Acc&& acc) {
    const size_t n = bl.size();
    // S_k = sum_{j>k} rgb_j alpha_j T_j + T_final * bg, built back to front
    double Ssuf[3] = {Tfin * bg[0], Tfin * bg[1], Tfin * bg[2]};
    for (size_t kk = n; kk-- > 0;) {
        const Blended& e = bl[kk];
        const Rec<double>& r = recs[e.g];
        G2* ap = acc(e.g);
        const double w = e.alpha * e.T;
        if (ap) {
            G2& a = *ap;
            double galpha = 0;
            for (int c = 0; c < 3; ++c) {
                a.rgb[c] += gbar[c] * w;
                galpha += gbar[c] * (r.rgb[c] * e.T - Ssuf[c] / (1.0 - e.alpha));
            }
            if (!e.clamped) {
                a.op += galpha * e.G;
                const double gpow = galpha * e.alpha;
                // power = -1/2 (Qa dx^2 + 2 Qb dx dy + Qc dy^2), dx = x - u, dy = y - v
                a.u += gpow * (r.Q[0] * e.dx + r.Q[1] * e.dy);
                a.v += gpow * (r.Q[1] * e.dx + r.Q[2] * e.dy);
                a.Q[0] += gpow * (-0.5 * e.dx * e.dx);
                a.Q[1] += gpow * (-e.dx * e.dy);
                a.Q[2] += gpow * (-0.5 * e.dy * e.dy);
            }
        }
        for (int c = 0; c < 3; ++c) Ssuf[c] += r.rgb[c] * w;
    }
}

// Full backward of one view: screen-space gradients g2[N] (accumulated, optional
// output) and per-parameter gradients (accumulated into grad).
void render_view_bwd(const OScene& sc, const OView& V, int B, const float* dimg, const OGrad& grad, double* g2out) {
    std::vector<Rec<double>> recs;
    preprocess_all<double>(sc, nullptr, V, recs);
    const int N = (int)recs.size();
    TileLists tl;
    build_tiles(N, V.W, V.H, B,
                [&](int g, int& x0, int& x1, int& y0, int& y1, float& key) {
                    const Rec<double>& r = recs[g];
                    if (!r.visible) return false;
                    x0 = r.x0; x1 = r.x1; y0 = r.y0; y1 = r.y1; key = r.key;
                    return true;
                },
                tl);
    const int T = tl.tx * tl.ty;
    const int HW = V.W * V.H;
    const int nth = omp_get_max_threads();
    std::vector<std::vector<G2>> acc(nth, std::vector<G2>((size_t)N, G2{0, 0, {0, 0, 0}, 0, {0, 0, 0}}));
#pragma omp parallel
    {
        std::vector<Blended> bl;
        std::vector<G2>& my = acc[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 4)
        for (int t = 0; t < T; ++t) {
            const int tx = t % tl.tx, ty = t / tl.tx;
            const int32_t* list = tl.ids.data() + tl.start[t];
            const int64_t len = tl.start[t + 1] - tl.start[t];
            for (int j = ty * B; j < std::min(V.H, (ty + 1) * B); ++j)
                for (int i = tx * B; i < std::min(V.W, (tx + 1) * B); ++i) {
                    bl.clear();
                    double C[3], Tp;
                    int nb;
                    bool a;
                    blend_pixel<double>(i, j, list, len, recs, V, C, Tp, nb, a, &bl);
                    const size_t p = (size_t)j * V.W + i;
                    const double gb[3] = {dimg[p], dimg[(size_t)HW + p], dimg[2 * (size_t)HW + p]};
                    blend_pixel_bwd(bl, recs, Tp, V.bg, gb, [&](int g) { return &my[g]; });
                }
        }
    }
    std::vector<G2> g2((size_t)N, G2{0, 0, {0, 0, 0}, 0, {0, 0, 0}});
    for (int th = 0; th < nth; ++th)
        for (int g = 0; g < N; ++g) {
            const G2& s = acc[th][g];
            G2& d = g2[g];
            d.u += s.u; d.v += s.v; d.op += s.op;
            for (int k = 0; k < 3; ++k) { d.Q[k] += s.Q[k]; d.rgb[k] += s.rgb[k]; }
        }
    if (g2out)
        for (int g = 0; g < N; ++g) {
            double* o = g2out + (size_t)9 * g;
            o[0] += g2[g].u; o[1] += g2[g].v;
            o[2] += g2[g].Q[0]; o[3] += g2[g].Q[1]; o[4] += g2[g].Q[2];
            o[5] += g2[g].op;
            o[6] += g2[g].rgb[0]; o[7] += g2[g].rgb[1]; o[8] += g2[g].rgb[2];
        }
    const int n4 = sc.n4, n3 = sc.n3;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < N; ++g) {
        if (!recs[g].visible) continue;
        double gmu[3] = {0, 0, 0}, gmt = 0, gls[4] = {0, 0, 0, 0}, gq[4] = {0, 0, 0, 0}, gq2[4] = {0, 0, 0, 0}, gop = 0,
               gsh[48], gsht[48 * kMaxTimeDeg];
        std::memset(gsh, 0, sizeof(gsh));
        std::memset(gsht, 0, sizeof(gsht));
        gaussian_bwd(sc, g, V, g2[g], gmu, &gmt, gls, gq, gq2, &gop, gsh, gsht);
        if (g < n4) {
            const size_t n = n4, i = g;
            if (grad.sht4)
                for (int k = 0; k < 48 * sc.sht_deg; ++k) grad.sht4[k * n + i] += gsht[k];
            for (int k = 0; k < 3; ++k) grad.mean4[k * n + i] += gmu[k];
            grad.mt4[i] += gmt;
            for (int k = 0; k < 4; ++k) grad.ls4[k * n + i] += gls[k];
            for (int k = 0; k < 4; ++k) grad.ql4[k * n + i] += gq[k];
            for (int k = 0; k < 4; ++k) grad.qr4[k * n + i] += gq2[k];
            grad.op4[i] += gop;
            for (int k = 0; k < 48; ++k) grad.sh4[k * n + i] += gsh[k];
        } else {
            const size_t n = n3, i = g - n4;
            for (int k = 0; k < 3; ++k) grad.mean3[k * n + i] += gmu[k];
            for (int k = 0; k < 3; ++k) grad.ls3[k * n + i] += gls[k];
            for (int k = 0; k < 4; ++k) grad.q3[k * n + i] += gq[k];
            grad.op3[i] += gop;
            for (int k = 0; k < 48; ++k) grad.sh3[k * n + i] += gsh[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Local evaluation around a few selected Gaussians of a large scene.
// A Gaussian's parameters change the image only inside its pixel square, so
// its gradient, and central differences of a loss that is linear in the image,
// need only the pixels of that square.  They are composited from the same
// depth-ordered candidate lists as the whole-view path, built here for the
// tiles the selected squares touch only, from every Gaussian's record.
// ---------------------------------------------------------------------------
constexpr int kRow = 65;  // one Gaussian's raw parameters in ABI field order (a 3D row uses the first 59)

// Parameter k of a Gaussian's row: 4D mean(3) mean_t log_scale(4) quat_l(4)
// quat_r(4) opacity sh(48); 3D mean(3) log_scale(3) quat(4) opacity sh(48).
inline double* param_slot(Param<double>& P, int k) {
    if (P.is4d) {
        if (k < 3) return &P.mu[k];
        if (k == 3) return &P.mt;
        if (k < 8) return &P.ls[k - 4];
        if (k < 12) return &P.q[k - 8];
        if (k < 16) return &P.q2[k - 12];
        if (k == 16) return &P.op;
        if (k < 65) return &P.sh[k - 17];
    } else {
        if (k < 3) return &P.mu[k];
        if (k < 6) return &P.ls[k - 3];
        if (k < 10) return &P.q[k - 6];
        if (k == 10) return &P.op;
        if (k < 59) return &P.sh[k - 11];
    }
    return nullptr;
}

// Record of Gaussian g in view V with parameter k moved by delta (k < 0: none).
inline Rec<double> record_of(const OScene& sc, const OView& V, int g, int k, double delta, double* theta = nullptr) {
    Param<double> P;
    load_param<double>(sc, nullptr, g, P);
    if (k >= 0) {
        double* x = param_slot(P, k);
        *x += delta;
        if (theta) *theta = *x;
    }
    Geo<double> G;
    world(P, V.time, G);
    Rec<double> r;
    project(V, P, G, r);
    return r;
}

// Records with one Gaussian's record replaced.
struct Overlay {
    const std::vector<Rec<double>>* base;
    int g;
    const Rec<double>* alt;
    const Rec<double>& operator[](size_t i) const { return (int)i == g ? *alt : (*base)[i]; }
};

inline bool has_square(const Rec<double>& r) { return r.r > 0 && r.x0 <= r.x1 && r.y0 <= r.y1; }

struct LocalView {
    OView V;
    int B = 16, tx = 0, ty = 0;
    std::vector<Rec<double>> recs;
    std::vector<int32_t> slot;                // tile -> index into lists, -1 when untouched
    std::vector<std::vector<int32_t>> lists;  // candidate lists of the touched tiles, (key, id) order
    std::vector<int32_t> region;              // pixels inside a selected square
    std::vector<uint8_t> amb;                 // per pixel of the view: guard-band flag (region pixels only)
    const int32_t* list_of(int i, int j, int64_t& len) const {
        const std::vector<int32_t>& l = lists[slot[(j / B) * tx + i / B]];
        len = (int64_t)l.size();
        return l.data();
    }
};

struct Local {
    OScene sc;
    std::vector<int32_t> sel;
    std::vector<int32_t> selidx;  // merged id -> selection index, -1 otherwise
    std::vector<LocalView> views;
};

// Records of every Gaussian, candidate lists of the tiles holding a pixel of
// `in_region` (one byte per pixel), and the guard-band flags of those pixels.
void local_build(const OScene& sc, const OView& V, int B, const std::vector<uint8_t>& in_region, LocalView& lv) {
    lv.V = V;
    lv.B = B;
    lv.tx = (V.W + B - 1) / B;
    lv.ty = (V.H + B - 1) / B;
    if (lv.recs.empty()) preprocess_all<double>(sc, nullptr, V, lv.recs);
    const int N = (int)lv.recs.size();
    const int T = lv.tx * lv.ty;
    lv.slot.assign(T, -1);
    int nl = 0;
    lv.region.clear();
    for (size_t p = 0; p < in_region.size(); ++p)
        if (in_region[p]) {
            lv.region.push_back((int32_t)p);
            const int t = (int)((p / V.W) / B) * lv.tx + (int)((p % V.W) / B);
            if (lv.slot[t] < 0) lv.slot[t] = nl++;
        }
    lv.lists.assign(nl, {});
    // per tile row, prefix counts of touched tiles: a Gaussian whose tile range
    // touches none is skipped without visiting its tiles
    std::vector<int32_t> pre((size_t)lv.ty * (lv.tx + 1), 0);
    for (int t2 = 0; t2 < lv.ty; ++t2)
        for (int t1 = 0; t1 < lv.tx; ++t1)
            pre[(size_t)t2 * (lv.tx + 1) + t1 + 1] = pre[(size_t)t2 * (lv.tx + 1) + t1] + (lv.slot[t2 * lv.tx + t1] >= 0);
    // the same candidates as the whole-view path: every Gaussian that is not
    // culled, over its square widened by one pixel, taken in (depth key, id)
    // order so that every list comes out sorted
    std::vector<int32_t> order;
    order.reserve((size_t)N);
    for (int g = 0; g < N; ++g)
        if (!lv.recs[g].culled) order.push_back(g);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (lv.recs[a].key != lv.recs[b].key) return lv.recs[a].key < lv.recs[b].key;
        return a < b;
    });
    for (int g : order) {
        const Rec<double>& r = lv.recs[g];
        const int x0 = std::max(0, r.x0 - 1), x1 = std::min(V.W - 1, r.x1 + 1);
        const int y0 = std::max(0, r.y0 - 1), y1 = std::min(V.H - 1, r.y1 + 1);
        if (x0 > x1 || y0 > y1) continue;
        for (int t2 = y0 / B; t2 <= y1 / B; ++t2) {
            const int32_t* row = pre.data() + (size_t)t2 * (lv.tx + 1);
            if (row[x1 / B + 1] == row[x0 / B]) continue;
            for (int t1 = x0 / B; t1 <= x1 / B; ++t1) {
                const int s = lv.slot[t2 * lv.tx + t1];
                if (s >= 0) lv.lists[s].push_back(g);
            }
        }
    }
    // guard-band flags of the region pixels, as the whole-view path sets them
    lv.amb.assign((size_t)V.W * V.H, 0);
    for (int g = 0; g < N; ++g) {
        const Rec<double>& r = lv.recs[g];
        if (r.margin >= kGlobalTol || r.r == 0) continue;
        const int xa = std::max(0, r.x0 - 1), xb = std::min(V.W - 1, r.x1 + 1);
        const int ya = std::max(0, r.y0 - 1), yb = std::min(V.H - 1, r.y1 + 1);
        for (int j = ya; j <= yb; ++j)
            for (int i = xa; i <= xb; ++i) lv.amb[(size_t)j * V.W + i] = 1;
    }
    const int64_t nr = (int64_t)lv.region.size();
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < nr; ++k) {
        const int p = lv.region[k], i = p % V.W, j = p / V.W;
        int64_t len;
        const int32_t* list = lv.list_of(i, j, len);
        double C[3], Tp;
        int nb;
        bool a;
        blend_pixel<double>(i, j, list, len, lv.recs, V, C, Tp, nb, a, nullptr);
        if (a) lv.amb[p] = 1;
    }
}

// The region of the selected Gaussians: the pixels of their squares.
void local_setup(const OScene& sc, const OView& V, int B, const std::vector<int32_t>& sel, LocalView& lv) {
    preprocess_all<double>(sc, nullptr, V, lv.recs);
    std::vector<uint8_t> in_region((size_t)V.W * V.H, 0);
    for (int g : sel) {
        const Rec<double>& r = lv.recs[g];
        if (!has_square(r)) continue;
        for (int j = r.y0; j <= r.y1; ++j)
            for (int i = r.x0; i <= r.x1; ++i) in_region[(size_t)j * V.W + i] = 1;
    }
    local_build(sc, V, B, in_region, lv);
}

// Upstream gradient of a pixel channel, zero at guard-band pixels.
inline double upstream(const LocalView& lv, const float* dimg, int p, int c) {
    return lv.amb[p] ? 0.0 : (double)dimg[(size_t)c * lv.V.W * lv.V.H + p];
}

// ---------------------------------------------------------------------------
// Eq. 9: quaternion of a 3x3 rotation block, with Shepperd's largest-component
// method where 1 + trace is too small for the printed formula (reading).
// ---------------------------------------------------------------------------
void mat2quat(const double R[3][3], double q[4]) {
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (1.0 + tr > 1e-6) {
        const double w = 0.5 * std::sqrt(1.0 + tr);
        q[0] = w;
        q[1] = (R[2][1] - R[1][2]) / (4 * w);
        q[2] = (R[0][2] - R[2][0]) / (4 * w);
        q[3] = (R[1][0] - R[0][1]) / (4 * w);
        return;
    }
    if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        const double x = 0.5 * std::sqrt(std::max(0.0, 1.0 + R[0][0] - R[1][1] - R[2][2]));
        q[1] = x;
        q[0] = (R[2][1] - R[1][2]) / (4 * x);
        q[2] = (R[0][1] + R[1][0]) / (4 * x);
        q[3] = (R[0][2] + R[2][0]) / (4 * x);
    } else if (R[1][1] >= R[2][2]) {
        const double y = 0.5 * std::sqrt(std::max(0.0, 1.0 - R[0][0] + R[1][1] - R[2][2]));
        q[2] = y;
        q[0] = (R[0][2] - R[2][0]) / (4 * y);
        q[1] = (R[0][1] + R[1][0]) / (4 * y);
        q[3] = (R[1][2] + R[2][1]) / (4 * y);
    } else {
        const double zz = 0.5 * std::sqrt(std::max(0.0, 1.0 - R[0][0] - R[1][1] + R[2][2]));
        q[3] = zz;
        q[0] = (R[1][0] - R[0][1]) / (4 * zz);
        q[1] = (R[0][2] + R[2][0]) / (4 * zz);
        q[2] = (R[1][2] + R[2][1]) / (4 * zz);
    }
}

void rot4_of(const float* ql_raw, const float* qr_raw, size_t n, size_t i, double R[4][4]) {
    double a[4], b[4], qa[4], qb[4];
    for (int k = 0; k < 4; ++k) { a[k] = ql_raw[k * n + i]; b[k] = qr_raw[k * n + i]; }
    normalize4(a, qa);
    normalize4(b, qb);
    double L[4][4], Rr[4][4];
    left_iso(qa, L);
    right_iso(qb, Rr);
    matmul<double, 4>(L, Rr, R);
}

}  // namespace orc

// ===========================================================================
// C ABI for ctypes.
// ===========================================================================
using namespace orc;

extern "C" {

int orc_num_threads() { return omp_get_max_threads(); }

// Forward render of one view.  img: [3][H][W], Tfin, nblend, amb: [H][W] (each may be null except img).
int orc_render(const OScene* sc, const OView* V, int B, double* img, double* Tfin, int32_t* nblend, uint8_t* amb) {
    if (!sc || !V || !img || B <= 0 || V->W <= 0 || V->H <= 0) return 1;
    render_view<double>(*sc, nullptr, *V, B, img, Tfin, nblend, amb);
    return 0;
}

// Forward-mode derivative of the image along tangent tg: dimg [3][H][W].
int orc_render_jvp(const OScene* sc, const OTangent* tg, const OView* V, int B, double* img, double* dimg) {
    if (!sc || !tg || !V || !dimg) return 1;
    const size_t n = (size_t)3 * V->W * V->H;
    std::vector<Dual> out(n);
    render_view<Dual>(*sc, tg, *V, B, out.data(), nullptr, nullptr, nullptr);
    for (size_t k = 0; k < n; ++k) {
        dimg[k] = out[k].d;
        if (img) img[k] = out[k].v;
    }
    return 0;
}

// Backward of one view; gradients are ACCUMULATED into grad (caller zeroes),
// g2 (optional, [N][9]: du dv dQ00 dQ01 dQ11 dop drgb) likewise.
int orc_render_bwd(const OScene* sc, const OView* V, int B, const float* dimg, const OGrad* grad, double* g2) {
    if (!sc || !V || !dimg || !grad) return 1;
    render_view_bwd(*sc, *V, B, dimg, *grad, g2);
    return 0;
}

// Per-Gaussian screen-space records of one view, [N][20] float64:
// visible culled u v depth Q00 Q01 Q11 op r g b radius x0 x1 y0 y1 key margin pt
int orc_project(const OScene* sc, const OView* V, double* out) {
    if (!sc || !V || !out) return 1;
    const int N = sc->n3 + sc->n4;
#pragma omp parallel for schedule(static)
    for (int g = 0; g < N; ++g) {
        Param<double> P;
        load_param<double>(*sc, nullptr, g, P);
        Geo<double> G;
        world(P, V->time, G);
        Rec<double> r;
        project(*V, P, G, r);
        double* o = out + (size_t)20 * g;
        o[0] = r.visible; o[1] = r.culled;
        o[2] = r.culled ? 0 : r.u; o[3] = r.culled ? 0 : r.v; o[4] = r.culled ? 0 : r.depth;
        for (int k = 0; k < 3; ++k) o[5 + k] = r.culled ? 0 : r.Q[k];
        o[8] = r.culled ? 0 : r.op;
        for (int k = 0; k < 3; ++k) o[9 + k] = r.culled ? 0 : r.rgb[k];
        o[12] = r.r; o[13] = r.x0; o[14] = r.x1; o[15] = r.y0; o[16] = r.y1;
        o[17] = r.key; o[18] = r.margin; o[19] = G.pt;
    }
    return 0;
}

// World-space stage of one Gaussian: mu[3], Sigma[9] (row-major), op, sig, pt.
int orc_world(const OScene* sc, int g, double time, double* mu, double* Sg, double* op3) {
    if (!sc || g < 0 || g >= sc->n3 + sc->n4) return 1;
    Param<double> P;
    load_param<double>(*sc, nullptr, g, P);
    Geo<double> G;
    world(P, time, G);
    for (int i = 0; i < 3; ++i) mu[i] = G.mu[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Sg[3 * i + j] = G.Sg[i][j];
    op3[0] = G.op; op3[1] = G.sig; op3[2] = G.pt;
    return 0;
}

// Eq. 4 pieces for checking: L, Rr, R = L Rr (all 4x4 row-major) of raw quaternions.
int orc_rot4(const double* ql, const double* qr, double* L, double* Rr, double* R) {
    double a[4], b[4];
    normalize4(ql, a);
    normalize4(qr, b);
    double Lm[4][4], Rm[4][4], P[4][4];
    left_iso(a, Lm);
    right_iso(b, Rm);
    matmul<double, 4>(Lm, Rm, P);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) { L[4 * i + j] = Lm[i][j]; Rr[4 * i + j] = Rm[i][j]; R[4 * i + j] = P[i][j]; }
    return 0;
}

int orc_quat_to_rot(const double* q, double* R) {
    double a[4], M[3][3];
    normalize4(q, a);
    quat_to_rot(a, M);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[3 * i + j] = M[i][j];
    return 0;
}

int orc_mat2quat(const double* R, double* q) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = R[3 * i + j];
    mat2quat(M, q);
    return 0;
}

// ---- local evaluation around selected Gaussians -----------------------------
// The scene arrays must stay alive until orc_local_free.  sel: merged ids
// (4D rows first), distinct.
void* orc_local_new(const OScene* sc, int n_views, const OView* views, int B, int n_sel, const int32_t* sel) {
    if (!sc || !views || n_views < 1 || B <= 0 || n_sel < 0) return nullptr;
    if (sc->sht_deg != 0) return nullptr;  // local rows hold no time coefficients
    const int N = sc->n3 + sc->n4;
    Local* L = new Local();
    L->sc = *sc;
    L->sel.assign(sel, sel + n_sel);
    L->selidx.assign((size_t)N, -1);
    for (int s = 0; s < n_sel; ++s) {
        if (sel[s] < 0 || sel[s] >= N || L->selidx[sel[s]] >= 0) { delete L; return nullptr; }
        L->selidx[sel[s]] = s;
    }
    L->views.resize(n_views);
    for (int v = 0; v < n_views; ++v) local_setup(*sc, views[v], B, L->sel, L->views[v]);
    return L;
}

void orc_local_free(void* h) { delete static_cast<Local*>(h); }

// The Gaussians blended at given pixels of one view, front to back, with their
// blend weights alpha T: ids / weights [npx][cap], counts[npx] (the full count,
// of which the first min(count, cap) are written).
int orc_blended_at(const OScene* sc, const OView* V, int B, int npx, const int32_t* px, const int32_t* py, int cap,
                   int32_t* ids, double* weights, int32_t* counts) {
    if (!sc || !V || B <= 0 || npx < 0 || cap < 0 || !px || !py || !counts) return 1;
    std::vector<uint8_t> in_region((size_t)V->W * V->H, 0);
    for (int k = 0; k < npx; ++k) {
        if (px[k] < 0 || px[k] >= V->W || py[k] < 0 || py[k] >= V->H) return 1;
        in_region[(size_t)py[k] * V->W + px[k]] = 1;
    }
    LocalView lv;
    local_build(*sc, *V, B, in_region, lv);
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < npx; ++k) {
        int64_t len;
        const int32_t* list = lv.list_of(px[k], py[k], len);
        std::vector<Blended> bl;
        double C[3], Tp;
        int nb;
        bool a;
        blend_pixel<double>(px[k], py[k], list, len, lv.recs, *V, C, Tp, nb, a, &bl);
        counts[k] = (int32_t)bl.size();
        for (int e = 0; e < std::min<int>(cap, (int)bl.size()); ++e) {
            ids[(size_t)k * cap + e] = bl[e].g;
            weights[(size_t)k * cap + e] = bl[e].alpha * bl[e].T;
        }
    }
    return 0;
}

// Per pixel of view v: bit 0 = inside a selected square, bit 1 = guard-band flag.
int orc_local_amb(void* h, int v, uint8_t* out) {
    const Local* L = static_cast<const Local*>(h);
    if (!L || v < 0 || v >= (int)L->views.size() || !out) return 1;
    const LocalView& lv = L->views[v];
    std::memset(out, 0, (size_t)lv.V.W * lv.V.H);
    for (int p : lv.region) out[p] = (uint8_t)(1 | (lv.amb[p] ? 2 : 0));
    return 0;
}

// Gradients of the selected Gaussians, summed over the views, of
// L = sum_v <dimgs[v], C_v> with dimgs zeroed at guard-band pixels:
// rows[n_sel][65] in the ABI field order (a 3D row fills its first 59).
int orc_local_grad(void* h, const float* const* dimgs, double* rows) {
    const Local* L = static_cast<const Local*>(h);
    if (!L || !dimgs || !rows) return 1;
    const int ns = (int)L->sel.size();
    std::fill(rows, rows + (size_t)ns * kRow, 0.0);
    const int nth = omp_get_max_threads();
    for (size_t v = 0; v < L->views.size(); ++v) {
        const LocalView& lv = L->views[v];
        const float* dimg = dimgs[v];
        std::vector<std::vector<G2>> acc(nth, std::vector<G2>((size_t)ns, G2{0, 0, {0, 0, 0}, 0, {0, 0, 0}}));
        const int64_t nr = (int64_t)lv.region.size();
#pragma omp parallel
        {
            std::vector<Blended> bl;
            std::vector<G2>& my = acc[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 64)
            for (int64_t k = 0; k < nr; ++k) {
                const int p = lv.region[k], i = p % lv.V.W, j = p / lv.V.W;
                int64_t len;
                const int32_t* list = lv.list_of(i, j, len);
                bl.clear();
                double C[3], Tp;
                int nb;
                bool a;
                blend_pixel<double>(i, j, list, len, lv.recs, lv.V, C, Tp, nb, a, &bl);
                const double gb[3] = {upstream(lv, dimg, p, 0), upstream(lv, dimg, p, 1), upstream(lv, dimg, p, 2)};
                blend_pixel_bwd(bl, lv.recs, Tp, lv.V.bg, gb, [&](int g) -> G2* {
                    const int s = L->selidx[g];
                    return s >= 0 ? &my[s] : nullptr;
                });
            }
        }
        for (int s = 0; s < ns; ++s) {
            const int g = L->sel[s];
            if (!lv.recs[g].visible) continue;
            G2 gs{0, 0, {0, 0, 0}, 0, {0, 0, 0}};
            for (int th = 0; th < nth; ++th) {
                const G2& a = acc[th][s];
                gs.u += a.u; gs.v += a.v; gs.op += a.op;
                for (int k = 0; k < 3; ++k) { gs.Q[k] += a.Q[k]; gs.rgb[k] += a.rgb[k]; }
            }
            double gmu[3] = {0, 0, 0}, gmt = 0, gls[4] = {0, 0, 0, 0}, gq[4] = {0, 0, 0, 0}, gq2[4] = {0, 0, 0, 0},
                   gop = 0, gsh[48];
            std::memset(gsh, 0, sizeof(gsh));
            gaussian_bwd(L->sc, g, lv.V, gs, gmu, &gmt, gls, gq, gq2, &gop, gsh, nullptr);
            double* o = rows + (size_t)s * kRow;
            if (g < L->sc.n4) {
                for (int k = 0; k < 3; ++k) o[k] += gmu[k];
                o[3] += gmt;
                for (int k = 0; k < 4; ++k) { o[4 + k] += gls[k]; o[8 + k] += gq[k]; o[12 + k] += gq2[k]; }
                o[16] += gop;
                for (int k = 0; k < 48; ++k) o[17 + k] += gsh[k];
            } else {
                for (int k = 0; k < 3; ++k) { o[k] += gmu[k]; o[3 + k] += gls[k]; }
                for (int k = 0; k < 4; ++k) o[6 + k] += gq[k];
                o[10] += gop;
                for (int k = 0; k < 48; ++k) o[11 + k] += gsh[k];
            }
        }
    }
    return 0;
}

// Central differences of the same loss: entry e moves parameter ent[2e + 1]
// of selected Gaussian ent[2e] by +-hrel max(1, |theta|) (in float64) and
// re-composites that Gaussian's square in every view.  ok[e] = 0 when either
// move changes a discrete decision: the Gaussian's cull, square, clamps or
// list position, or any pixel's blend count or clamped count (the loss is
// discontinuous or kinked there).  fd[e] = (L+ - L-) / (theta+ - theta-).
int orc_local_fd(void* h, const float* const* dimgs, int n_ent, const int32_t* ent, double hrel, double* fd,
                 int32_t* ok) {
    const Local* L = static_cast<const Local*>(h);
    if (!L || !dimgs || n_ent < 0 || !ent || !fd || !ok) return 1;
    auto nclamp = [](const std::vector<Blended>& b) {
        int c = 0;
        for (const Blended& x : b) c += x.clamped;
        return c;
    };
    // per (selected Gaussian, view): blend and clamp counts of the pixels of its
    // square at the unmoved parameters, computed on first use
    std::vector<std::vector<std::vector<int32_t>>> base(L->sel.size(), std::vector<std::vector<int32_t>>(L->views.size()));
    for (int e = 0; e < n_ent; ++e) {
        const int s = ent[2 * e], k = ent[2 * e + 1];
        fd[e] = 0.0;
        ok[e] = 0;
        if (s < 0 || s >= (int)L->sel.size()) return 1;
        const int g = L->sel[s];
        if (k < 0 || k >= (g < L->sc.n4 ? 65 : 59)) return 1;
        Param<double> P;
        load_param<double>(L->sc, nullptr, g, P);
        const double theta = *param_slot(P, k);
        const double step = hrel * std::max(1.0, std::fabs(theta));
        double tp = 0, tm = 0, dL = 0;
        bool same = true;
        for (size_t v = 0; v < L->views.size() && same; ++v) {
            const LocalView& lv = L->views[v];
            const Rec<double>& r0 = lv.recs[g];
            const Rec<double> rp = record_of(L->sc, lv.V, g, k, step, &tp);
            const Rec<double> rm = record_of(L->sc, lv.V, g, k, -step, &tm);
            for (const Rec<double>* r : {&rp, &rm})
                same = same && r->culled == r0.culled && r->visible == r0.visible && r->r == r0.r &&
                       r->x0 == r0.x0 && r->x1 == r0.x1 && r->y0 == r0.y0 && r->y1 == r0.y1 && r->kinks == r0.kinks;
            if (!same || !has_square(r0)) continue;
            // the depth order must keep g where it was in the lists of its tiles
            for (int t2 = r0.y0 / lv.B; t2 <= r0.y1 / lv.B && same; ++t2)
                for (int t1 = r0.x0 / lv.B; t1 <= r0.x1 / lv.B && same; ++t1) {
                    const std::vector<int32_t>& l = lv.lists[lv.slot[t2 * lv.tx + t1]];
                    const auto it = std::find(l.begin(), l.end(), g);
                    if (it == l.end()) continue;
                    for (const Rec<double>* r : {&rp, &rm}) {
                        if (it != l.begin()) {
                            const Rec<double>& q = lv.recs[*(it - 1)];
                            if (!(q.key < r->key || (q.key == r->key && *(it - 1) < g))) same = false;
                        }
                        if (it + 1 != l.end()) {
                            const Rec<double>& q = lv.recs[*(it + 1)];
                            if (!(r->key < q.key || (r->key == q.key && g < *(it + 1)))) same = false;
                        }
                    }
                }
            if (!same) break;
            const Overlay op{&lv.recs, g, &rp}, om{&lv.recs, g, &rm};
            const float* dimg = dimgs[v];
            const int W = lv.V.W, sw = r0.x1 - r0.x0 + 1;
            const int npx = sw * (r0.y1 - r0.y0 + 1);
            std::vector<int32_t>& b0 = base[s][v];
            if (b0.empty()) {
                b0.resize(2 * (size_t)npx);
#pragma omp parallel for schedule(dynamic, 64)
                for (int q = 0; q < npx; ++q) {
                    const int i = r0.x0 + q % sw, j = r0.y0 + q / sw;
                    int64_t len;
                    const int32_t* list = lv.list_of(i, j, len);
                    std::vector<Blended> b;
                    double C[3], T;
                    int n;
                    bool a;
                    blend_pixel<double>(i, j, list, len, lv.recs, lv.V, C, T, n, a, &b);
                    b0[2 * q] = n;
                    b0[2 * q + 1] = nclamp(b);
                }
            }
            double acc = 0.0;
            int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : acc, bad)
            for (int q = 0; q < npx; ++q) {
                const int i = r0.x0 + q % sw, j = r0.y0 + q / sw;
                const int p = j * W + i;
                int64_t len;
                const int32_t* list = lv.list_of(i, j, len);
                std::vector<Blended> b1, b2;
                double C1[3], C2[3], T1, T2;
                int n1, n2;
                bool a;
                blend_pixel<double, Overlay>(i, j, list, len, op, lv.V, C1, T1, n1, a, &b1);
                blend_pixel<double, Overlay>(i, j, list, len, om, lv.V, C2, T2, n2, a, &b2);
                if (n1 != b0[2 * q] || n2 != b0[2 * q] || nclamp(b1) != b0[2 * q + 1] || nclamp(b2) != b0[2 * q + 1])
                    ++bad;
                for (int c = 0; c < 3; ++c)
                    acc += upstream(lv, dimg, p, c) * ((C1[c] + T1 * lv.V.bg[c]) - (C2[c] + T2 * lv.V.bg[c]));
            }
            if (bad) same = false;
            dL += acc;
        }
        ok[e] = same ? 1 : 0;
        fd[e] = same && tp != tm ? dL / (tp - tm) : 0.0;
    }
    return 0;
}

int orc_sh_basis(const double* dir, double* Y) {
    sh_basis(dir, Y);
    return 0;
}

// Brute-force colour of selected pixels: every Gaussian tested, no tiles.
int orc_pixels(const OScene* sc, const OView* V, int npx, const int32_t* px, const int32_t* py, double* rgb,
               double* Tfin, uint8_t* amb) {
    if (!sc || !V) return 1;
    std::vector<Rec<double>> recs;
    preprocess_all<double>(*sc, nullptr, *V, recs);
    const int N = (int)recs.size();
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < npx; ++k) {
        const int i = px[k], j = py[k];
        std::vector<int32_t> cand;
        for (int g = 0; g < N; ++g) {
            const Rec<double>& r = recs[g];
            if (r.r == 0) continue;
            if (i < r.x0 - 1 || i > r.x1 + 1 || j < r.y0 - 1 || j > r.y1 + 1) continue;
            cand.push_back(g);
        }
        std::sort(cand.begin(), cand.end(), [&](int a, int b) {
            if (recs[a].key != recs[b].key) return recs[a].key < recs[b].key;
            return a < b;
        });
        double C[3], Tp;
        int nb;
        bool a;
        blend_pixel<double>(i, j, cand.data(), (int64_t)cand.size(), recs, *V, C, Tp, nb, a, nullptr);
        bool flagged = a;
        for (int g : cand) {
            const Rec<double>& r = recs[g];
            if (r.margin < kGlobalTol && r.r > 0) flagged = true;
        }
        for (int c = 0; c < 3; ++c) rgb[3 * k + c] = C[c] + Tp * V->bg[c];
        if (Tfin) Tfin[k] = Tp;
        if (amb) amb[k] = flagged;
    }
    return 0;
}

// Alg. 1 CreateTiles to IdentifyTileRanges on given screen-space splats (u, v, integer radius, depth
// key, visibility): exact tile lists.  First call with ids == null returns the
// pair count in *npairs; second call fills start[tiles+1] and ids[npairs].
int orc_tile_lists(int n, const float* u, const float* v, const int32_t* radius, const float* depth,
                   const uint8_t* visible, int W, int H, int B, int64_t* npairs, int64_t* start, int32_t* ids) {
    TileLists tl;
    build_tiles(n, W, H, B,
                [&](int g, int& x0, int& x1, int& y0, int& y1, float& key) {
                    if (!visible[g]) return false;
                    const double uu = u[g], vv = v[g];
                    const int r = radius[g];
                    x0 = std::max(0, (int)std::ceil(uu - r - 0.5));
                    x1 = std::min(W - 1, (int)std::floor(uu + r - 0.5));
                    y0 = std::max(0, (int)std::ceil(vv - r - 0.5));
                    y1 = std::min(H - 1, (int)std::floor(vv + r - 0.5));
                    key = depth[g];
                    return x0 <= x1 && y0 <= y1;
                },
                tl);
    *npairs = (int64_t)tl.ids.size();
    if (start) std::copy(tl.start.begin(), tl.start.end(), start);
    if (ids) std::copy(tl.ids.begin(), tl.ids.end(), ids);
    return 0;
}

// Alg. 1 CreateTiles to BlendInOrder on given screen-space splats: image [3][H][W] and T [H][W].
int orc_composite_records(int n, const float* u, const float* v, const float* conic /*[3][n]*/, const float* op,
                          const float* rgb /*[3][n]*/, const int32_t* radius, const float* depth,
                          const uint8_t* visible, int W, int H, int B, const double* bg, double* img, double* Tfin,
                          uint8_t* amb) {
    std::vector<Rec<double>> recs((size_t)n);
    for (int g = 0; g < n; ++g) {
        Rec<double>& r = recs[g];
        if (!visible[g]) { r.culled = true; continue; }
        r.culled = false;
        r.u = u[g]; r.v = v[g]; r.depth = depth[g]; r.key = depth[g];
        for (int k = 0; k < 3; ++k) { r.Q[k] = conic[(size_t)k * n + g]; r.rgb[k] = rgb[(size_t)k * n + g]; }
        r.op = op[g];
        r.r = radius[g];
        r.x0 = std::max(0, (int)std::ceil(r.u - r.r - 0.5));
        r.x1 = std::min(W - 1, (int)std::floor(r.u + r.r - 0.5));
        r.y0 = std::max(0, (int)std::ceil(r.v - r.r - 0.5));
        r.y1 = std::min(H - 1, (int)std::floor(r.v + r.r - 0.5));
        r.visible = r.x0 <= r.x1 && r.y0 <= r.y1;
        if (!r.visible) r.culled = true;
    }
    TileLists tl;
    build_tiles(n, W, H, B,
                [&](int g, int& x0, int& x1, int& y0, int& y1, float& key) {
                    const Rec<double>& r = recs[g];
                    if (r.culled) return false;
                    x0 = r.x0; x1 = r.x1; y0 = r.y0; y1 = r.y1; key = r.key;
                    return true;
                },
                tl);
    OView V{};
    V.W = W; V.H = H;
    for (int c = 0; c < 3; ++c) V.bg[c] = bg[c];
    const int HW = W * H;
    const int T = tl.tx * tl.ty;
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < T; ++t) {
        const int tx = t % tl.tx, ty = t / tl.tx;
        const int32_t* list = tl.ids.data() + tl.start[t];
        const int64_t len = tl.start[t + 1] - tl.start[t];
        for (int j = ty * B; j < std::min(H, (ty + 1) * B); ++j)
            for (int i = tx * B; i < std::min(W, (tx + 1) * B); ++i) {
                double C[3], Tp;
                int nb;
                bool a;
                blend_pixel<double>(i, j, list, len, recs, V, C, Tp, nb, a, nullptr);
                const size_t p = (size_t)j * W + i;
                for (int c = 0; c < 3; ++c) img[(size_t)c * HW + p] = C[c] + Tp * bg[c];
                if (Tfin) Tfin[p] = Tp;
                if (amb) amb[p] = a;
            }
    }
    return 0;
}

// Static identification and 4D->3D conversion (Sec. 4.1-4.2, Eq. 7-9).
// mask_i = (double)ls4[3][i] > log((double)tau) ("exceeds": strict).  Outputs:
// out4 rows = kept rows in order, out3 rows = in3 rows then converted rows in
// ascending 4D index; perm[i] = new 4D row, or -(1 + new 3D row).
// qout (float64, [4][n_conv]) is the Eq. 9 quaternion of each converted row.
int orc_convert_static(const OScene* sc, float tau, int32_t* perm, int32_t* n4_out, int32_t* n3_out, double* qout) {
    const size_t n4 = sc->n4;
    const double thr = std::log((double)tau);
    int32_t keep = 0, conv = 0;
    std::vector<int32_t> convrows;
    for (size_t i = 0; i < n4; ++i) {
        const bool m = (double)sc->ls4[3 * n4 + i] > thr;
        if (m) { perm[i] = -(1 + sc->n3 + conv); ++conv; convrows.push_back((int32_t)i); }
        else { perm[i] = keep; ++keep; }
    }
    *n4_out = keep;
    *n3_out = sc->n3 + conv;
    if (qout) {
        const size_t nc = convrows.size();
        for (size_t k = 0; k < nc; ++k) {
            double R[4][4], R3[3][3], q[4];
            rot4_of(sc->ql4, sc->qr4, n4, (size_t)convrows[k], R);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) R3[i][j] = R[i][j];
            mat2quat(R3, q);
            for (int c = 0; c < 4; ++c) qout[c * nc + k] = q[c];
        }
    }
    return 0;
}

// One Adam step (Kingma & Ba) in float64 on float32 inputs, bias-corrected.
int orc_adam(int64_t n, const float* p, const float* g, const float* m, const float* v, double lr, double b1,
             double b2, double eps, int step, double* p_out, double* m_out, double* v_out) {
    const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        const double mm = b1 * m[i] + (1.0 - b1) * g[i];
        const double vv = b2 * v[i] + (1.0 - b2) * (double)g[i] * g[i];
        m_out[i] = mm;
        v_out[i] = vv;
        p_out[i] = p[i] - lr * (mm / c1) / (std::sqrt(vv / c2) + eps);
    }
    return 0;
}

}  // extern "C"

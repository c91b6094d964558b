// Adaptive densification and pruning on gfx950, applied to the static 3D and
// the dynamic 4D set separately (Sec. 4.3, which adopts the clone / split /
// prune scheme of 3D Gaussian Splatting): per row a selection from the
// accumulated image-plane gradient, clone or split by the largest spatial
// scale, prune by opacity and size; then three stable compactions (kept
// originals, clones, split children) and a scatter of the output rows.
// Decisions compare float32 values widened to double against double limits,
// so they are exact; split children are placed in FP64.
#include "common.hpp"
#include "launch.hpp"
#include "rotation.hpp"

namespace h4d {

struct RowFlags {
    bool keep_orig, keep_clone, keep_child;
};

// Decisions of one row.  ls: its log-scales (nls of them; the first three are
// spatial); opacity: its logit.
__device__ inline RowFlags densify_row(const DensifyP& p, float grad, float vis, const float* ls, int nls,
                                       float opacity) {
    const bool sel = vis > 0.0f && (double)grad >= (double)p.thr * (double)vis;
    double L = (double)ls[0], Lc = (double)(float)((double)ls[0] - p.log_shrink);
    for (int k = 1; k < 3; ++k) {
        L = fmax(L, (double)ls[k]);
        Lc = fmax(Lc, (double)(float)((double)ls[k] - p.log_shrink));
    }
    (void)nls;
    const bool large = L > p.log_dense;
    const bool low = (double)opacity < p.logit_min;
    const bool pr = low || L > p.log_max_scale;
    const bool prc = low || Lc > p.log_max_scale;
    RowFlags f;
    f.keep_orig = !(sel && large) && !pr;
    f.keep_clone = sel && !large && !pr;
    f.keep_child = sel && large && !prc;
    return f;
}

__global__ void k_densify_flags3(G3Ptr g, const float* __restrict__ grad, const float* __restrict__ vis, DensifyP p,
                                 uint32_t* __restrict__ f0, uint32_t* __restrict__ f1, uint32_t* __restrict__ f2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const size_t n = (size_t)g.n;
    float ls[3];
    for (int k = 0; k < 3; ++k) ls[k] = g.log_scale[k * n + i];
    const RowFlags f = densify_row(p, grad[i], vis[i], ls, 3, g.opacity[i]);
    f0[i] = f.keep_orig; f1[i] = f.keep_clone; f2[i] = f.keep_child;
}

__global__ void k_densify_flags4(G4Ptr g, const float* __restrict__ grad, const float* __restrict__ vis, DensifyP p,
                                 uint32_t* __restrict__ f0, uint32_t* __restrict__ f1, uint32_t* __restrict__ f2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const size_t n = (size_t)g.n;
    float ls[4];
    for (int k = 0; k < 4; ++k) ls[k] = g.log_scale[k * n + i];
    const RowFlags f = densify_row(p, grad[i], vis[i], ls, 4, g.opacity[i]);
    f0[i] = f.keep_orig; f1[i] = f.keep_clone; f2[i] = f.keep_child;
}

// Output position of each kind: kept originals first, then clones, then the
// children, child k of every split row after child k - 1 of all of them.
// sc: the three exclusive scans [3][n + 1].
struct DensifyPos {
    const unsigned long long* s0;
    const unsigned long long* s1;
    const unsigned long long* s2;
};

__device__ inline void copy_row3(const G3Ptr& g, size_t i, const G3Grad& o, size_t r) {
    const size_t n = (size_t)g.n, no = (size_t)o.n;
    for (int k = 0; k < 3; ++k) o.mean[k * no + r] = g.mean[k * n + i];
    for (int k = 0; k < 3; ++k) o.log_scale[k * no + r] = g.log_scale[k * n + i];
    for (int k = 0; k < 4; ++k) o.quat[k * no + r] = g.quat[k * n + i];
    o.opacity[r] = g.opacity[i];
    for (int k = 0; k < 48; ++k) o.sh[k * no + r] = g.sh[k * n + i];
}

__device__ inline void copy_row4(const G4Ptr& g, size_t i, const G4Grad& o, size_t r) {
    const size_t n = (size_t)g.n, no = (size_t)o.n;
    for (int k = 0; k < 3; ++k) o.mean[k * no + r] = g.mean[k * n + i];
    o.mean_t[r] = g.mean_t[i];
    for (int k = 0; k < 4; ++k) o.log_scale[k * no + r] = g.log_scale[k * n + i];
    for (int k = 0; k < 4; ++k) o.quat_l[k * no + r] = g.quat_l[k * n + i];
    for (int k = 0; k < 4; ++k) o.quat_r[k * no + r] = g.quat_r[k * n + i];
    o.opacity[r] = g.opacity[i];
    for (int k = 0; k < 48; ++k) o.sh[k * no + r] = g.sh[k * n + i];
    if (g.sh_t)
        for (int k = 0; k < 48 * g.sh_t_deg; ++k) o.sh_t[k * no + r] = g.sh_t[k * n + i];
}

// noise: [split_n][3][n] standard normal draws
__global__ void k_densify_scatter3(G3Ptr g, DensifyPos ps, const float* __restrict__ noise, DensifyP p, G3Grad o,
                                   int32_t* __restrict__ src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)g.n;
    if (i >= g.n) return;
    const unsigned long long K0 = ps.s0[n], K1 = ps.s1[n], K2 = ps.s2[n];
    const bool k0 = ps.s0[i + 1] != ps.s0[i], k1 = ps.s1[i + 1] != ps.s1[i], k2 = ps.s2[i + 1] != ps.s2[i];
    if (k0) {
        const size_t r = ps.s0[i];
        copy_row3(g, i, o, r);
        src[r] = i;
    }
    if (k1) {
        const size_t r = K0 + ps.s1[i];
        copy_row3(g, i, o, r);
        src[r] = -1 - i;
    }
    if (k2) {
        double q[4], R[3][3], s[3];
        load_unit4(g.quat, g.n, i, q);
        quat_rot3(q, R);
        for (int k = 0; k < 3; ++k) s[k] = exp((double)g.log_scale[k * n + i]);
        const size_t no = (size_t)o.n;
        for (int c = 0; c < p.split_n; ++c) {
            const size_t r = K0 + K1 + (size_t)c * K2 + ps.s2[i];
            copy_row3(g, i, o, r);
            double z[3];
            for (int k = 0; k < 3; ++k) z[k] = s[k] * (double)noise[((size_t)c * 3 + k) * n + i];
            for (int a = 0; a < 3; ++a)
                o.mean[a * no + r] = (float)((double)g.mean[a * n + i] + R[a][0] * z[0] + R[a][1] * z[1] +
                                             R[a][2] * z[2]);
            for (int k = 0; k < 3; ++k) o.log_scale[k * no + r] = (float)((double)g.log_scale[k * n + i] - p.log_shrink);
            src[r] = -1 - i;
        }
    }
}

// noise: [split_n][4][n]; children move in space and time along R_l R_r (Eq. 4)
__global__ void k_densify_scatter4(G4Ptr g, DensifyPos ps, const float* __restrict__ noise, DensifyP p, G4Grad o,
                                   int32_t* __restrict__ src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)g.n;
    if (i >= g.n) return;
    const unsigned long long K0 = ps.s0[n], K1 = ps.s1[n], K2 = ps.s2[n];
    const bool k0 = ps.s0[i + 1] != ps.s0[i], k1 = ps.s1[i + 1] != ps.s1[i], k2 = ps.s2[i + 1] != ps.s2[i];
    if (k0) {
        const size_t r = ps.s0[i];
        copy_row4(g, i, o, r);
        src[r] = i;
    }
    if (k1) {
        const size_t r = K0 + ps.s1[i];
        copy_row4(g, i, o, r);
        src[r] = -1 - i;
    }
    if (k2) {
        double ql[4], qr[4], L[4][4], Rr[4][4], R[4][4], s[4];
        load_unit4(g.quat_l, g.n, i, ql);
        load_unit4(g.quat_r, g.n, i, qr);
        rot_left(ql, L);
        rot_right(qr, Rr);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += L[a][k] * Rr[k][b];
                R[a][b] = acc;
            }
        for (int k = 0; k < 4; ++k) s[k] = exp((double)g.log_scale[k * n + i]);
        const size_t no = (size_t)o.n;
        for (int c = 0; c < p.split_n; ++c) {
            const size_t r = K0 + K1 + (size_t)c * K2 + ps.s2[i];
            copy_row4(g, i, o, r);
            double z[4], d[4];
            for (int k = 0; k < 4; ++k) z[k] = s[k] * (double)noise[((size_t)c * 4 + k) * n + i];
            for (int a = 0; a < 4; ++a) d[a] = R[a][0] * z[0] + R[a][1] * z[1] + R[a][2] * z[2] + R[a][3] * z[3];
            for (int a = 0; a < 3; ++a) o.mean[a * no + r] = (float)((double)g.mean[a * n + i] + d[a]);
            o.mean_t[r] = (float)((double)g.mean_t[i] + d[3]);
            for (int k = 0; k < 4; ++k) o.log_scale[k * no + r] = (float)((double)g.log_scale[k * n + i] - p.log_shrink);
            src[r] = -1 - i;
        }
    }
}

__global__ void k_densify_count(DensifyPos ps, int n, int split_n, int32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *out = (int32_t)(ps.s0[n] + ps.s1[n] + (unsigned long long)split_n * ps.s2[n]);
}

// Rows of the optimiser state after densification: out row r takes in row
// src[r] (src >= 0) or zeros (a new row).
__global__ void k_gather_rows3(G3Ptr g, const int32_t* __restrict__ src, int rows, G3Grad o) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int32_t i = src[r];
    const size_t n = (size_t)g.n, no = (size_t)o.n;
    auto get = [&](const float* a, int k) { return (i >= 0 && (size_t)i < n) ? a[k * n + i] : 0.0f; };
    for (int k = 0; k < 3; ++k) o.mean[k * no + r] = get(g.mean, k);
    for (int k = 0; k < 3; ++k) o.log_scale[k * no + r] = get(g.log_scale, k);
    for (int k = 0; k < 4; ++k) o.quat[k * no + r] = get(g.quat, k);
    o.opacity[r] = get(g.opacity, 0);
    for (int k = 0; k < 48; ++k) o.sh[k * no + r] = get(g.sh, k);
}

__global__ void k_gather_rows4(G4Ptr g, const int32_t* __restrict__ src, int rows, G4Grad o) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const int32_t i = src[r];
    const size_t n = (size_t)g.n, no = (size_t)o.n;
    auto get = [&](const float* a, int k) { return (i >= 0 && (size_t)i < n) ? a[k * n + i] : 0.0f; };
    for (int k = 0; k < 3; ++k) o.mean[k * no + r] = get(g.mean, k);
    o.mean_t[r] = get(g.mean_t, 0);
    for (int k = 0; k < 4; ++k) o.log_scale[k * no + r] = get(g.log_scale, k);
    for (int k = 0; k < 4; ++k) o.quat_l[k * no + r] = get(g.quat_l, k);
    for (int k = 0; k < 4; ++k) o.quat_r[k * no + r] = get(g.quat_r, k);
    o.opacity[r] = get(g.opacity, 0);
    for (int k = 0; k < 48; ++k) o.sh[k * no + r] = get(g.sh, k);
    if (g.sh_t)
        for (int k = 0; k < 48 * g.sh_t_deg; ++k) o.sh_t[k * no + r] = get(g.sh_t, k);
}

namespace {
DensifyPos scans_of(unsigned long long* scan, int n) {
    return DensifyPos{scan, scan + (n + 1), scan + 2 * (size_t)(n + 1)};
}
}  // namespace

void launch_densify3(const G3Ptr& g, const float* grad, const float* vis, const float* noise, const DensifyP& p,
                     const G3Grad& o, int32_t* src, uint32_t* flags, unsigned long long* scan,
                     unsigned long long* partials, int32_t* count, hipStream_t st) {
    const int n = g.n;
    const int nb = std::max(1, scan_blocks(n));
    if (n > 0) k_densify_flags3<<<ceil_div(n, 256), 256, 0, st>>>(g, grad, vis, p, flags, flags + n, flags + 2 * n);
    for (int k = 0; k < 3; ++k)
        launch_scan_u32_u64(flags + (size_t)k * n, nullptr, n, scan + (size_t)k * (n + 1),
                            partials + (size_t)k * (nb + 1), st);
    const DensifyPos ps = scans_of(scan, n);
    if (n > 0) k_densify_scatter3<<<ceil_div(n, 256), 256, 0, st>>>(g, ps, noise, p, o, src);
    k_densify_count<<<1, 1, 0, st>>>(ps, n, p.split_n, count);
}

void launch_densify4(const G4Ptr& g, const float* grad, const float* vis, const float* noise, const DensifyP& p,
                     const G4Grad& o, int32_t* src, uint32_t* flags, unsigned long long* scan,
                     unsigned long long* partials, int32_t* count, hipStream_t st) {
    const int n = g.n;
    const int nb = std::max(1, scan_blocks(n));
    if (n > 0) k_densify_flags4<<<ceil_div(n, 256), 256, 0, st>>>(g, grad, vis, p, flags, flags + n, flags + 2 * n);
    for (int k = 0; k < 3; ++k)
        launch_scan_u32_u64(flags + (size_t)k * n, nullptr, n, scan + (size_t)k * (n + 1),
                            partials + (size_t)k * (nb + 1), st);
    const DensifyPos ps = scans_of(scan, n);
    if (n > 0) k_densify_scatter4<<<ceil_div(n, 256), 256, 0, st>>>(g, ps, noise, p, o, src);
    k_densify_count<<<1, 1, 0, st>>>(ps, n, p.split_n, count);
}

void launch_gather_rows(const G3Ptr& g3, const int32_t* src3, int rows3, const G3Grad& o3, const G4Ptr& g4,
                        const int32_t* src4, int rows4, const G4Grad& o4, hipStream_t st) {
    if (rows3 > 0) k_gather_rows3<<<ceil_div(rows3, 256), 256, 0, st>>>(g3, src3, rows3, o3);
    if (rows4 > 0) k_gather_rows4<<<ceil_div(rows4, 256), 256, 0, st>>>(g4, src4, rows4, o4);
}

}  // namespace h4d

// Static identification and 4D -> 3D conversion on gfx950 (Sec. 4.1-4.2,
// Eq. 7-9): mask, stable compaction of the 4D set, append of the converted rows
// to the 3D set with the Eq. 9 quaternion of the spatial rotation block.  A
// converted row keeps its time-independent SH coefficients; its time
// coefficients (if any) are dropped with the time axis.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

// mask_i = (double)s_t > log((double)tau); flags hold 1 for converted rows
__global__ void k_convert_mask(const float* __restrict__ ls4, int n4, double log_tau, uint32_t* __restrict__ conv,
                               uint32_t* __restrict__ keep) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const bool m = (double)ls4[(size_t)3 * n4 + i] > log_tau;
    conv[i] = m ? 1u : 0u;
    keep[i] = m ? 0u : 1u;
}

__device__ inline void mat2quat(const double R[3][3], double q[4]) {
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (1.0 + tr > 1e-6) {
        const double w = 0.5 * sqrt(1.0 + tr);
        const double i4w = 1.0 / (4.0 * w);
        q[0] = w;
        q[1] = (R[2][1] - R[1][2]) * i4w;
        q[2] = (R[0][2] - R[2][0]) * i4w;
        q[3] = (R[1][0] - R[0][1]) * i4w;
        return;
    }
    // largest-diagonal branch (Shepperd) where the printed formula degenerates
    if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        const double x = 0.5 * sqrt(fmax(0.0, 1.0 + R[0][0] - R[1][1] - R[2][2]));
        const double i4 = 1.0 / (4.0 * x);
        q[1] = x; q[0] = (R[2][1] - R[1][2]) * i4; q[2] = (R[0][1] + R[1][0]) * i4; q[3] = (R[0][2] + R[2][0]) * i4;
    } else if (R[1][1] >= R[2][2]) {
        const double y = 0.5 * sqrt(fmax(0.0, 1.0 - R[0][0] + R[1][1] - R[2][2]));
        const double i4 = 1.0 / (4.0 * y);
        q[2] = y; q[0] = (R[0][2] - R[2][0]) * i4; q[1] = (R[0][1] + R[1][0]) * i4; q[3] = (R[1][2] + R[2][1]) * i4;
    } else {
        const double z = 0.5 * sqrt(fmax(0.0, 1.0 - R[0][0] - R[1][1] + R[2][2]));
        const double i4 = 1.0 / (4.0 * z);
        q[3] = z; q[0] = (R[1][0] - R[0][1]) * i4; q[1] = (R[0][2] + R[2][0]) * i4; q[2] = (R[1][2] + R[2][1]) * i4;
    }
}

__device__ inline void unit4(const float* q, int n, int i, double o[4]) {
    double a[4];
    for (int k = 0; k < 4; ++k) a[k] = (double)q[(size_t)k * n + i];
    const double inv = 1.0 / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3]);
    for (int k = 0; k < 4; ++k) o[k] = a[k] * inv;
}

// keep_off / conv_off: exclusive scans of keep / conv (64-bit), [n4 + 1]
__global__ void k_convert_scatter(G4Ptr in4, const uint32_t* __restrict__ conv,
                                  const unsigned long long* __restrict__ keep_off,
                                  const unsigned long long* __restrict__ conv_off, int n3, G4Grad out4, G3Grad out3,
                                  int32_t* __restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n4 = in4.n;
    if (i >= n4) return;
    const size_t ni = (size_t)n4;
    if (!conv[i]) {
        const size_t r = (size_t)keep_off[i];
        const size_t no = (size_t)out4.n;  // output capacity (row stride)
        for (int k = 0; k < 3; ++k) out4.mean[k * no + r] = in4.mean[k * ni + i];
        out4.mean_t[r] = in4.mean_t[i];
        for (int k = 0; k < 4; ++k) out4.log_scale[k * no + r] = in4.log_scale[k * ni + i];
        for (int k = 0; k < 4; ++k) out4.quat_l[k * no + r] = in4.quat_l[k * ni + i];
        for (int k = 0; k < 4; ++k) out4.quat_r[k * no + r] = in4.quat_r[k * ni + i];
        out4.opacity[r] = in4.opacity[i];
        for (int k = 0; k < 48; ++k) out4.sh[k * no + r] = in4.sh[k * ni + i];
        if (in4.sh_t)
            for (int k = 0; k < 48 * in4.sh_t_deg; ++k) out4.sh_t[k * no + r] = in4.sh_t[k * ni + i];
        perm[i] = (int32_t)r;
    } else {
        const size_t r = (size_t)n3 + (size_t)conv_off[i];
        const size_t no = (size_t)out3.n;
        for (int k = 0; k < 3; ++k) out3.mean[k * no + r] = in4.mean[k * ni + i];
        for (int k = 0; k < 3; ++k) out3.log_scale[k * no + r] = in4.log_scale[k * ni + i];
        out3.opacity[r] = in4.opacity[i];
        for (int k = 0; k < 48; ++k) out3.sh[k * no + r] = in4.sh[k * ni + i];
        // Eq. 8-9: quaternion of the top-left 3x3 block of R_l R_r
        double a[4], b[4];
        unit4(in4.quat_l, n4, i, a);
        unit4(in4.quat_r, n4, i, b);
        const double L[4][4] = {{a[0], -a[1], -a[2], -a[3]}, {a[1], a[0], -a[3], a[2]},
                                {a[2], a[3], a[0], -a[1]}, {a[3], -a[2], a[1], a[0]}};
        const double Rr[4][4] = {{b[0], -b[1], -b[2], -b[3]}, {b[1], b[0], b[3], -b[2]},
                                 {b[2], -b[3], b[0], b[1]}, {b[3], b[2], -b[1], b[0]}};
        double R3[3][3];
        for (int r2 = 0; r2 < 3; ++r2)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int k = 0; k < 4; ++k) acc += L[r2][k] * Rr[k][c];
                R3[r2][c] = acc;
            }
        double q[4];
        mat2quat(R3, q);
        for (int k = 0; k < 4; ++k) out3.quat[k * no + r] = (float)q[k];
        perm[i] = -(int32_t)(1 + r);
    }
}

// copy of the existing 3D rows into the (wider) output arrays
__global__ void k_copy_rows(G3Ptr in3, G3Grad out3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= in3.n) return;
    const size_t ni = (size_t)in3.n, no = (size_t)out3.n;
    for (int k = 0; k < 3; ++k) out3.mean[k * no + i] = in3.mean[k * ni + i];
    for (int k = 0; k < 3; ++k) out3.log_scale[k * no + i] = in3.log_scale[k * ni + i];
    for (int k = 0; k < 4; ++k) out3.quat[k * no + i] = in3.quat[k * ni + i];
    out3.opacity[i] = in3.opacity[i];
    for (int k = 0; k < 48; ++k) out3.sh[k * no + i] = in3.sh[k * ni + i];
}

__global__ void k_convert_counts(const unsigned long long* keep_off, const unsigned long long* conv_off, int n4, int n3,
                                 int32_t* counts) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        counts[0] = (int32_t)keep_off[n4];
        counts[1] = n3 + (int32_t)conv_off[n4];
    }
}

// Optimiser state across the conversion: the moment arrays (laid out as the
// parameters) follow the rows the conversion moved (perm from
// k_convert_scatter).  A kept 4D row takes all its moments; a converted row
// takes those of the fields it copies (mean, spatial log-scales, opacity, SH)
// and starts its new quaternion's at zero.
__global__ void k_convert_moments(G4Ptr in4, const int32_t* __restrict__ perm, G4Grad out4, G3Grad out3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n4 = in4.n;
    if (i >= n4) return;
    const size_t ni = (size_t)n4;
    const int32_t p = perm[i];
    if (p >= 0) {
        const size_t r = (size_t)p, no = (size_t)out4.n;
        for (int k = 0; k < 3; ++k) out4.mean[k * no + r] = in4.mean[k * ni + i];
        out4.mean_t[r] = in4.mean_t[i];
        for (int k = 0; k < 4; ++k) out4.log_scale[k * no + r] = in4.log_scale[k * ni + i];
        for (int k = 0; k < 4; ++k) out4.quat_l[k * no + r] = in4.quat_l[k * ni + i];
        for (int k = 0; k < 4; ++k) out4.quat_r[k * no + r] = in4.quat_r[k * ni + i];
        out4.opacity[r] = in4.opacity[i];
        for (int k = 0; k < 48; ++k) out4.sh[k * no + r] = in4.sh[k * ni + i];
        if (in4.sh_t)
            for (int k = 0; k < 48 * in4.sh_t_deg; ++k) out4.sh_t[k * no + r] = in4.sh_t[k * ni + i];
    } else {
        const size_t r = (size_t)(-1 - (int64_t)p), no = (size_t)out3.n;
        for (int k = 0; k < 3; ++k) out3.mean[k * no + r] = in4.mean[k * ni + i];
        for (int k = 0; k < 3; ++k) out3.log_scale[k * no + r] = in4.log_scale[k * ni + i];
        for (int k = 0; k < 4; ++k) out3.quat[k * no + r] = 0.0f;
        out3.opacity[r] = in4.opacity[i];
        for (int k = 0; k < 48; ++k) out3.sh[k * no + r] = in4.sh[k * ni + i];
    }
}

void launch_convert_moments(const G4Ptr& in4, const G3Ptr& in3, const int32_t* perm, const G4Grad& out4,
                            const G3Grad& out3, hipStream_t st) {
    if (in3.n > 0) k_copy_rows<<<ceil_div(in3.n, 256), 256, 0, st>>>(in3, out3);
    if (in4.n > 0) k_convert_moments<<<ceil_div(in4.n, 256), 256, 0, st>>>(in4, perm, out4, out3);
}

// flags: [2][n4] uint32; scan: [2][n4 + 1] u64; partials: [2][scan_blocks + 1]
void launch_convert_static(const G4Ptr& in4, const G3Ptr& in3, double log_tau, const G4Grad& out4,
                           const G3Grad& out3, int32_t* perm, uint32_t* flags, unsigned long long* scan,
                           unsigned long long* partials, int32_t* counts, hipStream_t st) {
    const int n4 = in4.n;
    uint32_t* conv = flags;
    uint32_t* keep = flags + n4;
    unsigned long long* conv_off = scan;
    unsigned long long* keep_off = scan + (n4 + 1);
    const int nb = std::max(1, scan_blocks(n4));
    if (in3.n > 0) k_copy_rows<<<ceil_div(in3.n, 256), 256, 0, st>>>(in3, out3);
    if (n4 > 0) k_convert_mask<<<ceil_div(n4, 256), 256, 0, st>>>(in4.log_scale, n4, log_tau, conv, keep);
    launch_scan_u32_u64(conv, nullptr, n4, conv_off, partials, st);
    launch_scan_u32_u64(keep, nullptr, n4, keep_off, partials + nb + 1, st);
    if (n4 > 0)
        k_convert_scatter<<<ceil_div(n4, 256), 256, 0, st>>>(in4, conv, keep_off, conv_off, in3.n, out4, out3, perm);
    k_convert_counts<<<1, 1, 0, st>>>(keep_off, conv_off, n4, in3.n, counts);
}

}  // namespace h4d

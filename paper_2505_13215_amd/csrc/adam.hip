// Bias-corrected Adam over several float32 segments in one launch.
// HBM-bound: 16 B read + 12 B written per scalar; float4 vectorised when a
// segment is 16-byte aligned and a multiple of 4 long, scalar otherwise.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, const AdamTable& t) {
    const float b1 = t.b1, b2 = t.b2, eps = t.eps, c1 = t.c1, c2 = t.c2;
    m = b1 * m + t.omb1 * g;
    v = b2 * v + t.omb2 * g * g;
    const float mh = m / c1, vh = v / c2;
    p -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void __launch_bounds__(256) k_adam(AdamTable t) {
    const AdamSeg& s = t.seg[blockIdx.y];
    const bool vec = ((reinterpret_cast<uintptr_t>(s.p) | reinterpret_cast<uintptr_t>(s.g) |
                       reinterpret_cast<uintptr_t>(s.m) | reinterpret_cast<uintptr_t>(s.v)) & 15u) == 0 &&
                     (s.n & 3) == 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    if (vec) {
        float4* P = reinterpret_cast<float4*>(s.p);
        const float4* G = reinterpret_cast<const float4*>(s.g);
        float4* M = reinterpret_cast<float4*>(s.m);
        float4* Vv = reinterpret_cast<float4*>(s.v);
        const size_t n4 = (size_t)s.n / 4;
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
            float4 p = P[i], m = M[i], v = Vv[i];
            const float4 g = G[i];
            adam_one(p.x, g.x, m.x, v.x, s.lr, t);
            adam_one(p.y, g.y, m.y, v.y, s.lr, t);
            adam_one(p.z, g.z, m.z, v.z, s.lr, t);
            adam_one(p.w, g.w, m.w, v.w, s.lr, t);
            P[i] = p; M[i] = m; Vv[i] = v;
        }
    } else {
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)s.n; i += stride) {
            float p = s.p[i], m = s.m[i], v = s.v[i];
            adam_one(p, s.g[i], m, v, s.lr, t);
            s.p[i] = p; s.m[i] = m; s.v[i] = v;
        }
    }
}

void launch_adam(const AdamTable& t, hipStream_t st) {
    if (t.n_seg <= 0) return;
    int64_t mx = 0;
    for (int i = 0; i < t.n_seg; ++i) mx = std::max(mx, t.seg[i].n);
    if (mx == 0) return;
    const int bx = (int)std::min<int64_t>(1024, (mx / 4 + 255) / 256 + 1);
    k_adam<<<dim3(bx, t.n_seg), 256, 0, st>>>(t);
}

}  // namespace h4d

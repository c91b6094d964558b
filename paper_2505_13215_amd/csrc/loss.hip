// L1 photometric loss and its gradient (elementwise, HBM-bound: 12 bytes per
// pixel channel).  Each thread keeps four 16-byte loads of each input in flight.
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

__device__ __forceinline__ float l1_sign(float d, float scale) { return d > 0.f ? scale : (d < 0.f ? -scale : 0.f); }

__device__ __forceinline__ float block_sum_256(float v) {
    __shared__ float s[4];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    return s[0] + s[1] + s[2] + s[3];
}

// n4 float4 groups (images are 16-byte aligned); the last n - 4 n4 scalars are
// handled by block 0.
__global__ void __launch_bounds__(256) k_l1_loss_grad(const float* __restrict__ img, const float* __restrict__ target,
                                                      float* __restrict__ dl, size_t n, float scale, float* loss) {
    const size_t n4 = n / 4;
    const float4* __restrict__ a4 = reinterpret_cast<const float4*>(img);
    const float4* __restrict__ b4 = reinterpret_cast<const float4*>(target);
    float4* __restrict__ o4 = reinterpret_cast<float4*>(dl);
    float acc = 0.f;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        float4 a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = a4[i + u * stride];
            b[u] = b4[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float dx = a[u].x - b[u].x, dy = a[u].y - b[u].y, dz = a[u].z - b[u].z, dw = a[u].w - b[u].w;
            o4[i + u * stride] = make_float4(l1_sign(dx, scale), l1_sign(dy, scale), l1_sign(dz, scale),
                                             l1_sign(dw, scale));
            acc += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
        }
    }
    for (; i < n4; i += stride) {
        const float4 a = a4[i], b = b4[i];
        const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, dw = a.w - b.w;
        o4[i] = make_float4(l1_sign(dx, scale), l1_sign(dy, scale), l1_sign(dz, scale), l1_sign(dw, scale));
        acc += fabsf(dx) + fabsf(dy) + fabsf(dz) + fabsf(dw);
    }
    if (blockIdx.x == 0) {
        for (size_t r = 4 * n4 + threadIdx.x; r < n; r += blockDim.x) {
            const float d = img[r] - target[r];
            dl[r] = l1_sign(d, scale);
            acc += fabsf(d);
        }
    }
    if (loss) {
        const float s = block_sum_256(acc);
        if (threadIdx.x == 0) atomicAdd(loss, s * scale);
    }
}

void launch_l1_loss_grad(const float* img, const float* target, float* dl, size_t n, float scale, float* loss,
                         hipStream_t st) {
    if (n == 0) return;
    const size_t n4 = n / 4;
    // one block per compute unit at most: the blocks end with an atomic on one
    // word, which serialises
    const int nb = (int)std::max<size_t>(1, std::min<size_t>(256, (n4 + 4 * 256 - 1) / (4 * 256)));
    k_l1_loss_grad<<<nb, 256, 0, st>>>(img, target, dl, n, scale, loss);
}

}  // namespace h4d

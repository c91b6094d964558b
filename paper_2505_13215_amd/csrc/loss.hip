// L1 photometric loss and its gradient (elementwise, HBM-bound).
#include "common.hpp"
#include "launch.hpp"

namespace h4d {

__global__ void __launch_bounds__(256) k_l1_loss_grad(const float* __restrict__ img, const float* __restrict__ target,
                                                      float* __restrict__ dl, size_t n, float scale, float* loss) {
    float acc = 0.f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = img[i] - target[i];
        dl[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
        acc += fabsf(d);
    }
    if (loss) {
        __shared__ float s[256];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) atomicAdd(loss, s[0] * scale);
    }
}

void launch_l1_loss_grad(const float* img, const float* target, float* dl, size_t n, float scale, float* loss,
                         hipStream_t st) {
    if (n == 0) return;
    const int nb = (int)std::min<size_t>(2048, (n + 255) / 256);
    k_l1_loss_grad<<<nb, 256, 0, st>>>(img, target, dl, n, scale, loss);
}

}  // namespace h4d

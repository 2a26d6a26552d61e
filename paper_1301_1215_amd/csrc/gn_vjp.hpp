// Kernels of the implicit derivative of a regularised Gauss-Newton step
// (Eq. 3, the linearisation point held fixed): complex a x + b y, FP64
// partial dot products summed in a fixed order, and the gradient with
// respect to the real sampling weights P.
#pragma once
#include <hip/hip_runtime.h>

#include "cg_scalars.hpp"
#include "fft_core.hpp"

namespace nlinv {

constexpr int kDotBlocks = 512;   // partial dot products per vector part

// z = a x + b y (x or y null: 0)
__global__ __launch_bounds__(kThreads) void k_axpby(float2* z, float a, const float2* x, float b, const float2* y,
                                                   long long n) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const float2 u = x ? x[i] : make_float2(0.f, 0.f);
        const float2 v = y ? y[i] : make_float2(0.f, 0.f);
        z[i] = make_float2(a * u.x + b * v.x, a * u.y + b * v.y);
    }
}

// partial[blockIdx.x] = sum over the block's stride of Re(conj(x) y), FP64
__global__ __launch_bounds__(kThreads) void k_dot_re(const float2* x, const float2* y, long long n, double* partial) {
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const float2 u = x[i], v = y[i];
        acc += (double)u.x * v.x + (double)u.y * v.y;
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out = scale * sum_{i < count} partial[i], in order (one thread)
__global__ void k_sum_partials(const double* partial, int count, double scale, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < count; ++i) s += partial[i];
    *out = scale * s;
}

// gP[k] = Re sum_j conj(u_j[k]) (y_j[k] - 2 P[k] w_j[k])
__global__ __launch_bounds__(kThreads) void k_gn_grad_P(const float2* u, const float2* y, const float2* w,
                                                       const float* P, float* gP, int J, long long N) {
    for (long long k = (long long)blockIdx.x * kThreads + threadIdx.x; k < N; k += (long long)gridDim.x * kThreads) {
        const float p2 = 2.f * P[k];
        float s = 0.f;
        for (int j = 0; j < J; ++j) {
            const float2 a = u[(long long)j * N + k], b = y[(long long)j * N + k], c = w[(long long)j * N + k];
            const float2 d = make_float2(b.x - p2 * c.x, b.y - p2 * c.y);
            s += a.x * d.x + a.y * d.y;
        }
        gP[k] = s;
    }
}

}  // namespace nlinv

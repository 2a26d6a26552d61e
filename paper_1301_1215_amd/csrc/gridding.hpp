// Gridding of radial k-space samples onto the Cartesian grid and its
// adjoint (Sec. 3.1: the measured non-Cartesian data are interpolated to
// the grid before the reconstruction; Sec. 3.2: on a grid doubled for the
// interpolation's accuracy), by convolution with a separable Kaiser-Bessel
// window:
//   samples   spoke s at angle th_s carries R samples at radii r_i = i - floor(R/2),
//             position k_si = (n/2 + r_i cos th_s, n/2 + r_i sin th_s) in grid units;
//   window    phi(d0, d1) = kb(d0) kb(d1), kb(d) = I0(beta sqrt(1 - (2d/W)^2)) / I0(beta)
//             for |d| <= W/2, else 0;
//   gridding  out[j][u][v] = sum_{s,i} dcf_i data[j][s][i] phi(u' - k0_si, v' - k1_si)
//             over the grid points u' = u (mod n), v' = v (mod n) within W/2 of the sample;
//   adjoint   data[j][s][i] = dcf_i sum phi(u' - k0_si, v' - k1_si) grid[j][u' mod n][v' mod n].
// Both are gathers (each output written by one thread, a fixed order), so
// the results do not depend on scheduling.  Positions, the test whether a
// grid point lies in a sample's window and the window itself are evaluated
// in FP64; the sums over samples are FP32.
#pragma once
#include <hip/hip_runtime.h>

#include "fft_core.hpp"

namespace nlinv {

constexpr int kGridCoilChunk = 8;    // coils per thread
constexpr int kMaxSpokes = 1024;     // spokes per call (angles staged in LDS)

struct GridArgs {
    int n, J, S, R;
    const float* angles;   // [S] radians
    const float* dcf;      // [R] density compensation per radius (nullable: 1)
    double width, beta;
    const float2* data;    // [J][S][R] (gridding input / degridding output)
    float2* out;           // gridding: [J][n][n]; degridding: [J][S][R]
    const float2* grid;    // degridding input [J][n][n]
};

// I0(x) = sum_k (x^2/4)^k / (k!)^2, summed until the terms no longer change
// the sum (FP64; x <= 40 needs < 80 terms)
__device__ __forceinline__ double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double s = 1.0, term = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        s += term;
        if (term < 1e-17 * s) break;
    }
    return s;
}

// kb(d) * I0(beta): the window without its normalisation (|d| <= W/2 holds)
__device__ __forceinline__ double kb_unnorm(double d, double width, double beta) {
    const double t = 1.0 - (2.0 * d / width) * (2.0 * d / width);
    return bessel_i0(beta * sqrt(t > 0.0 ? t : 0.0));
}

// Stage the spokes' directions (FP64) in LDS; returns 1/I0(beta)
__device__ __forceinline__ double stage_spokes(const GridArgs& g, double* cs, double* sn) {
    for (int s = threadIdx.x; s < g.S; s += blockDim.x) {
        const double th = (double)g.angles[s];
        cs[s] = cos(th);
        sn[s] = sin(th);
    }
    __syncthreads();
    return 1.0 / bessel_i0(g.beta);
}

// Radii r (as reals) with |a - r c| <= h; [lo, hi] empty when lo > hi
__device__ __forceinline__ void radius_interval(double a, double c, double h, double& lo, double& hi) {
    if (c > 0.0) {
        lo = (a - h) / c;
        hi = (a + h) / c;
    } else if (c < 0.0) {
        lo = (a + h) / c;
        hi = (a - h) / c;
    } else if (fabs(a) <= h) {
        lo = -1e300;
        hi = 1e300;
    } else {
        lo = 1.0;
        hi = -1.0;
    }
}

// Gridding: one thread per grid point (u, v) and chunk of kGridCoilChunk coils
__global__ __launch_bounds__(kThreads) void k_grid_radial(GridArgs g) {
    __shared__ double cs[kMaxSpokes], sn[kMaxSpokes];
    const double inv_i0b = stage_spokes(g, cs, sn);
    const long long e = (long long)blockIdx.x * kThreads + threadIdx.x;
    const long long nn = (long long)g.n * g.n;
    if (e >= nn) return;
    const int u = (int)(e / g.n), v = (int)(e % g.n);
    const int j0 = blockIdx.y * kGridCoilChunk;
    const int jn = min(kGridCoilChunk, g.J - j0);
    const double h = 0.5 * g.width, half = 0.5 * (double)g.n, eps = 1e-9;
    const int rhalf = g.R / 2;
    float2 acc[kGridCoilChunk];
    for (int j = 0; j < kGridCoilChunk; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int s = 0; s < g.S; ++s) {
        const double c = cs[s], d = sn[s];
        // the grid point and its copies one period away (windows that cross
        // the grid's edge wrap around)
        for (int du = -1; du <= 1; ++du) {
            const double idx0 = (double)(u + du * g.n);
            double lo0, hi0;
            radius_interval(idx0 - half, c, h, lo0, hi0);
            if (lo0 > hi0) continue;
            for (int dv = -1; dv <= 1; ++dv) {
                const double idx1 = (double)(v + dv * g.n);
                double lo1, hi1;
                radius_interval(idx1 - half, d, h, lo1, hi1);
                const double lo = fmax(lo0, lo1) - eps, hi = fmin(hi0, hi1) + eps;
                if (lo > hi) continue;
                const int ia = max(0, (int)ceil(fmax(lo, -1e9)) + rhalf);
                const int ib = min(g.R - 1, (int)floor(fmin(hi, 1e9)) + rhalf);
                for (int i = ia; i <= ib; ++i) {
                    const double r = (double)(i - rhalf);
                    const double k0 = half + r * c, k1 = half + r * d;
                    // the window's extent exactly as a sample's grid range
                    if (!(k0 - h <= idx0 && idx0 <= k0 + h && k1 - h <= idx1 && idx1 <= k1 + h)) continue;
                    double w = kb_unnorm(idx0 - k0, g.width, g.beta) * kb_unnorm(idx1 - k1, g.width, g.beta) *
                               inv_i0b * inv_i0b;
                    if (g.dcf) w *= (double)g.dcf[i];
                    const float wf = (float)w;
                    const float2* src = g.data + ((long long)j0 * g.S + s) * g.R + i;
                    for (int j = 0; j < jn; ++j) {
                        const float2 x = src[(long long)j * g.S * g.R];
                        acc[j].x += wf * x.x;
                        acc[j].y += wf * x.y;
                    }
                }
            }
        }
    }
    for (int j = 0; j < jn; ++j) g.out[(long long)(j0 + j) * nn + e] = acc[j];
}

// Degridding (the adjoint): one thread per sample (s, i) and chunk of coils
__global__ __launch_bounds__(kThreads) void k_degrid_radial(GridArgs g) {
    __shared__ double cs[kMaxSpokes], sn[kMaxSpokes];
    const double inv_i0b = stage_spokes(g, cs, sn);
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= g.S * g.R) return;
    const int s = e / g.R, i = e % g.R;
    const int j0 = blockIdx.y * kGridCoilChunk;
    const int jn = min(kGridCoilChunk, g.J - j0);
    const double h = 0.5 * g.width, half = 0.5 * (double)g.n;
    const double r = (double)(i - g.R / 2);
    const double k0 = half + r * cs[s], k1 = half + r * sn[s];
    const int a0 = (int)ceil(k0 - h), b0 = (int)floor(k0 + h);
    const int a1 = (int)ceil(k1 - h), b1 = (int)floor(k1 + h);
    const long long nn = (long long)g.n * g.n;
    float2 acc[kGridCoilChunk];
    for (int j = 0; j < kGridCoilChunk; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int x0 = a0; x0 <= b0; ++x0) {
        const double w0 = kb_unnorm((double)x0 - k0, g.width, g.beta) * inv_i0b;
        const int u = ((x0 % g.n) + g.n) % g.n;
        for (int x1 = a1; x1 <= b1; ++x1) {
            const float wf = (float)(w0 * kb_unnorm((double)x1 - k1, g.width, g.beta) * inv_i0b);
            const int v = ((x1 % g.n) + g.n) % g.n;
            const float2* src = g.grid + (long long)j0 * nn + (long long)u * g.n + v;
            for (int j = 0; j < jn; ++j) {
                const float2 y = src[(long long)j * nn];
                acc[j].x += wf * y.x;
                acc[j].y += wf * y.y;
            }
        }
    }
    const float d = g.dcf ? g.dcf[i] : 1.0f;
    for (int j = 0; j < jn; ++j)
        g.out[((long long)(j0 + j) * g.S + s) * g.R + i] = make_float2(d * acc[j].x, d * acc[j].y);
}

}  // namespace nlinv

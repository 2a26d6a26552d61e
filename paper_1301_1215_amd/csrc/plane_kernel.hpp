// The normal operator (DF^H DF + alpha) of Eq. 3 for one coil plane with the
// whole n x n plane held in LDS (small grids): one workgroup per plane runs
// all four centred 2D transforms of DF and DF^H in LDS and touches HBM only
// for its operands and results, instead of the five axis passes with their
// intermediates in HBM.  The rho part (the sum over the coils) is the fixed-
// order coil sum of coil_sum.hpp over the per-coil products this kernel
// writes.
#pragma once
#include <hip/hip_runtime.h>

#include "pass_kernels.hpp"

namespace nlinv {

struct PlaneArgs {
    const float2* rho;      // [m][m]     the linearisation point's image
    const float2* c;        // [planes][m][m] its coil maps c_j = E^H W^{-1} chat_j
    const float* P;         // [n][n]     sampling weights (row-major)
    const float* winv;      // [n][n]     1/w
    const float2* drho;     // [m][m]     direction, image part
    const float2* dchat;    // [planes][n][n] direction, sensitivity part
    float2* dchat_out;      // [planes][n][n] W^{-H} E(conj(rho) v_j) + alpha dchat_j
    float2* aux;            // [planes][m][m] conj(c_j) v_j (summed over j by the coil sum)
    const float2* tw2;      // [N1][N2] twiddles of the line split
    float alpha;
    float rs;               // 1/sqrt(n)
    int m, lo;              // Omega: rows and columns [lo, lo + m)
    int nplanes;
};

// Whole-plane kernels exist for grids whose plane and exchange buffer fit a
// workgroup's LDS next to a second workgroup.
constexpr bool plane_kernel_size(int n) { return n >= 8 && n <= 64; }
constexpr int plane_threads(int n) {
    const int n1 = split_n1(n), n2 = n / n1;
    const int t = n * (n1 > n2 ? n1 : n2);      // one stage task per thread
    const int r = ((t + 63) / 64) * 64;
    return r < 256 ? 256 : (r > 1024 ? 1024 : r);
}

// Line transforms of the plane A (row-major N x N, true positions) along one
// axis (AXIS 0: the columns, line = column and position = row; AXIS 1: the
// rows), in the two register stages of the line split N = N1 x N2 around the
// exchange buffer B.  B is line-fastest for the columns ([k1][j2][line]:
// adjacent threads take adjacent columns, adjacent LDS words) and
// [line][k1][j2] (padded) for the rows.  Every thread of the workgroup calls
// each stage; the caller puts the barriers between stages.
template <int N, int AXIS>
struct PlaneLines {
    using CT = Centre<N>;
    static constexpr int N1 = CT::N1, N2 = CT::N2, S2 = N2 + 1;
    static constexpr int BSIZE = N * N1 * S2;
    static __device__ __forceinline__ int bidx(int line, int k1, int j2) {
        return AXIS == 0 ? (k1 * N2 + j2) * N + line : (line * N1 + k1) * S2 + j2;
    }
    // tasks (line, j2) and (line, k1)
    static __device__ __forceinline__ void task_j2(int t, int& line, int& j2) {
        line = AXIS == 0 ? t % N : t / N2;
        j2 = AXIS == 0 ? t / N : t % N2;
    }
    static __device__ __forceinline__ void task_k1(int t, int& line, int& k1) {
        line = AXIS == 0 ? t % N : t / N1;
        k1 = AXIS == 0 ? t / N : t % N1;
    }
    // stage 1: x(line, in_pos) -> N1-point DFT -> twiddle -> B
    template <bool INV, int NT, class Get>
    static __device__ __forceinline__ void first(float2* B, const float2* TW, Get&& get) {
        for (int t = threadIdx.x; t < N * N2; t += NT) {
            int line, j2;
            task_j2(t, line, j2);
            float2 v[N1];
            static_for<0, N1>([&](auto K) {
                const int p = CT::in_pos(j2, K);
                v[K] = cscale(get(line, p), CT::sign(p));
            });
            RegDFT<N1, INV>::run(v);
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                float2 x = v[k1];
                if constexpr (k1 > 0) x = INV ? cmulc(x, TW[k1 * N2 + j2]) : cmul(x, TW[k1 * N2 + j2]);
                B[bidx(line, k1, j2)] = x;
            });
        }
    }
    // stage 2: B -> N2-point DFT -> put(line, out_pos, value times scale)
    template <bool INV, int NT, class Put>
    static __device__ __forceinline__ void second(const float2* B, float scale, Put&& put) {
        for (int t = threadIdx.x; t < N * N1; t += NT) {
            int line, k1;
            task_k1(t, line, k1);
            float2 v[N2];
            static_for<0, N2>([&](auto J) { v[J] = B[bidx(line, k1, J)]; });
            RegDFT<N2, INV>::run(v);
            static_for<0, N2>([&](auto K) {
                const int p = CT::out_pos(k1, K);
                put(line, p, cscale(v[K], CT::sign(p) * scale));
            });
        }
    }
    // stage 2 of one direction, the pointwise map f(line, pos, value) on the
    // true values (times rs), and the first stage of the other direction as
    // the adjoint of this stage 2, all on the task's registers, back into the
    // same slots of B
    template <bool INV_FIRST, int NT, class F>
    static __device__ __forceinline__ void middle(float2* B, float rs, F&& f) {
        for (int t = threadIdx.x; t < N * N1; t += NT) {
            int line, k1;
            task_k1(t, line, k1);
            float2 v[N2];
            static_for<0, N2>([&](auto J) { v[J] = B[bidx(line, k1, J)]; });
            RegDFT<N2, INV_FIRST>::run(v);
            static_for<0, N2>([&](auto K) {
                const int p = CT::out_pos(k1, K);
                const float sg = CT::sign(p);
                v[K] = cscale(f(line, p, cscale(v[K], sg * rs)), sg);
            });
            RegDFT<N2, !INV_FIRST>::run(v);
            static_for<0, N2>([&](auto J) { B[bidx(line, k1, J)] = v[J]; });
        }
    }
    // the adjoint of stage 1: twiddle, N1-point DFT, put(line, in_pos, value times rs)
    template <bool INV, int NT, class Put>
    static __device__ __forceinline__ void last(const float2* B, const float2* TW, float rs, Put&& put) {
        for (int t = threadIdx.x; t < N * N2; t += NT) {
            int line, j2;
            task_j2(t, line, j2);
            float2 v[N1];
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                v[k1] = B[bidx(line, k1, j2)];
                if constexpr (k1 > 0) v[k1] = INV ? cmulc(v[k1], TW[k1 * N2 + j2]) : cmul(v[k1], TW[k1 * N2 + j2]);
            });
            RegDFT<N1, INV>::run(v);
            static_for<0, N1>([&](auto K) {
                const int p = CT::in_pos(j2, K);
                put(line, p, cscale(v[K], CT::sign(p) * rs));
            });
        }
    }
};

// One coil plane: the columns' inverse transform of W^{-1} dchat from HBM;
// along the rows the inverse, z = c drho + rho dc on Omega and the forward
// transform (one fused step); along the columns the forward, P^2 and the
// inverse; along the rows the inverse, conj(c) v (to HBM) and conj(rho) v,
// and the forward; the columns' forward transform with W^{-H} and alpha dchat
// to HBM.  Each fused step is stage 1 | stage 2, pointwise, adjoint stage 2 |
// adjoint stage 1, with a barrier at each bar.
template <int N>
__global__ __launch_bounds__(plane_threads(N)) void k_plane_normal(PlaneArgs a) {
    constexpr int NT = plane_threads(N);
    using Col = PlaneLines<N, 0>;
    using Row = PlaneLines<N, 1>;
    static_assert(plane_kernel_size(N), "whole-plane size");
    __shared__ float2 A[N * N];
    __shared__ float2 B[Col::BSIZE];
    __shared__ float2 TW[N];
    const int plane = blockIdx.x;
    if (plane >= a.nplanes) return;
    const int m = a.m, lo = a.lo;
    const float rs = a.rs;
    const long long pb = (long long)plane * N * N, cb = (long long)plane * m * m;
    const float2* dchat = a.dchat + pb;
    const float2* c = a.c + cb;
    for (int e = threadIdx.x; e < N; e += NT) TW[e] = a.tw2[e];
    __syncthreads();
    auto in_om = [&](int i, int k) { return (unsigned)(i - lo) < (unsigned)m && (unsigned)(k - lo) < (unsigned)m; };
    auto colA = [&](int col, int row) -> float2& { return A[row * N + col]; };
    auto rowA = [&](int row, int col) -> float2& { return A[row * N + col]; };
    // dc_j = E^H W^{-1} dchat_j: the columns' inverse transform, from HBM
    Col::template first<true, NT>(B, TW, [&](int col, int row) { return cscale(dchat[row * N + col], a.winv[row * N + col]); });
    __syncthreads();
    Col::template second<true, NT>(B, rs, [&](int col, int row, float2 v) { colA(col, row) = v; });
    __syncthreads();
    // rows: inverse, z = c_j drho + rho dc_j on Omega (zero outside), forward
    Row::template first<true, NT>(B, TW, [&](int row, int col) { return rowA(row, col); });
    __syncthreads();
    Row::template middle<true, NT>(B, rs, [&](int row, int col, float2 dc) {
        if (!in_om(row, col)) return make_float2(0.f, 0.f);
        const int q = (row - lo) * m + (col - lo);
        return cadd(cmul(c[q], a.drho[q]), cmul(a.rho[q], dc));
    });
    __syncthreads();
    Row::template last<false, NT>(B, TW, rs, [&](int row, int col, float2 v) { rowA(row, col) = v; });
    __syncthreads();
    // columns: forward, P^2 (the sampling and its adjoint), inverse
    Col::template first<false, NT>(B, TW, [&](int col, int row) { return colA(col, row); });
    __syncthreads();
    Col::template middle<false, NT>(B, rs, [&](int col, int row, float2 x) {
        const float p = a.P[row * N + col];
        return cscale(x, p * p);
    });
    __syncthreads();
    Col::template last<true, NT>(B, TW, rs, [&](int col, int row, float2 v) { colA(col, row) = v; });
    __syncthreads();
    // rows: inverse, aux = conj(c_j) v_j and conj(rho) v_j on Omega, forward
    Row::template first<true, NT>(B, TW, [&](int row, int col) { return rowA(row, col); });
    __syncthreads();
    Row::template middle<true, NT>(B, rs, [&](int row, int col, float2 v) {
        if (!in_om(row, col)) return make_float2(0.f, 0.f);
        const int q = (row - lo) * m + (col - lo);
        a.aux[cb + q] = cconjmul(c[q], v);
        return cconjmul(a.rho[q], v);
    });
    __syncthreads();
    Row::template last<false, NT>(B, TW, rs, [&](int row, int col, float2 v) { rowA(row, col) = v; });
    __syncthreads();
    // columns: forward; W^{-H} E(conj(rho) v_j) + alpha dchat_j to HBM
    Col::template first<false, NT>(B, TW, [&](int col, int row) { return colA(col, row); });
    __syncthreads();
    Col::template second<false, NT>(B, rs, [&](int col, int row, float2 v) {
        const int e = row * N + col;
        const float2 d = dchat[e];
        const float2 x = cscale(v, a.winv[e]);
        a.dchat_out[pb + e] = make_float2(x.x + a.alpha * d.x, x.y + a.alpha * d.y);
    });
}

}  // namespace nlinv

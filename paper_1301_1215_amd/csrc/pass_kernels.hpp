// Fused pass kernels of the NLINV operators (Schaetz & Uecker, Eqs. 2-3)
// and the CG vector / FP64 reduction kernels, for gfx950.
//
// Data layout in HBM (complex64 interleaved, C-contiguous):
//   coil planes  [planes][n][n]   chat-like vectors and k-space data
//   Omega planes [planes][m][m]   sensitivities c_j restricted to Omega
//   image        [frames][m][m]   rho-like vectors
//   T            [planes][m][n]   intermediate between a column pass and a
//                                 row pass: only the m rows of Omega are kept
// A "plane" is one coil of one frame; plane_frame[] maps planes to frames of
// a shape class (all frames of a class share n and m).
//
// A 2D centred unitary DFT is a column pass (transform along axis 0) and a
// row pass (axis 1).  Along one axis, the centred DFT is an ordinary DFT
// between two checkerboard signs (-1)^index, times 1/sqrt(n); the global sign
// (-1)^(n/2) of each axis cancels between the two axes of a square grid.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace nlinv {

__device__ __forceinline__ float sgn(int i) { return (i & 1) ? -1.0f : 1.0f; }

// 1/w = (1 + a |k|^2)^(-l/2), k_d = (kappa_d - n/2)/n, evaluated in the log domain
// (w reaches 5e32 at the grid corners for a = 220, l = 32).
__device__ __forceinline__ float winv(int r, int c, int n, float a, float hl) {
    const int d0 = r - n / 2, d1 = c - n / 2;
    const float k2 = (float)(d0 * d0 + d1 * d1) / (float)(n * n);
    return expf(-hl * log1pf(a * k2));
}

// ---------------------------------------------------------------------------
// column passes: a workgroup transforms L adjacent columns of one plane
// ---------------------------------------------------------------------------

enum ColMode : int {
    COL_WINV_IFFT_CROP = 0,   // T = crop_rows(IDFT_0(chat / w))
    COL_P_IFFT_CROP = 1,      // T = crop_rows(IDFT_0(P . z))
    COL_PAD_FFT_P = 2,        // out = P . DFT_0(pad_rows(T))
    COL_PAD_FFT_P_RESID = 3,  // out = s_f y - P . DFT_0(pad_rows(T))
    COL_PAD_FFT_P2_IFFT = 4,  // T = crop_rows(IDFT_0(P^2 . DFT_0(pad_rows(T))))   (in place)
    COL_PAD_FFT_WINV_ADD = 5, // out = DFT_0(pad_rows(T)) / w + a1_f add1 + a2_f add2
    COL_PAD_FFT_GPROD = 6,    // outR = Re(conj(g) . DFT_0(pad_rows(T)))  (mask gradient)
};

struct ColArgs {
    const float2* in;
    float2* out;
    const float2* add1;       // RESID: y; WINV_ADD: first added vector; GPROD: g
    const float2* add2;
    const float* P;           // [frames][n][n] with stride p_stride (0 = shared)
    long long p_stride;
    const int* plane_frame;   // nullable: all planes in frame 0
    const float* s1;          // per-frame multiplier of add1 (nullable -> c1)
    const float* s2;
    float c1, c2;
    int m, lo;
    float sob_a, sob_hl;
    float rs;                 // 1/sqrt(n)
    const float2* tw;         // exp(-2 pi i k / n), k < n
};

template <int N, int L, int MODE>
__global__ __launch_bounds__(kThreads) void k_col(ColArgs a) {
    __shared__ float2 tile[N * L];
    __shared__ float2 tw[N];
    const int plane = blockIdx.y;
    const int col0 = blockIdx.x * L;
    const int f = a.plane_frame ? a.plane_frame[plane] : 0;
    const int m = a.m, lo = a.lo;
    for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = a.tw[i];

    constexpr bool IN_CROP = (MODE >= COL_PAD_FFT_P);
    constexpr bool INV1 = (MODE == COL_WINV_IFFT_CROP || MODE == COL_P_IFFT_CROP);
    const float* P = a.P + (long long)f * a.p_stride;

    if constexpr (IN_CROP) {
        const float2* src = a.in + (long long)plane * m * N;
        for (int idx = threadIdx.x; idx < N * L; idx += kThreads) {
            const int r = idx / L, c = idx % L;
            const int ri = r - lo;
            float2 v = make_float2(0.f, 0.f);
            if (ri >= 0 && ri < m) v = cscale(src[(long long)ri * N + col0 + c], sgn(r));
            tile[idx] = v;
        }
    } else {
        const float2* src = a.in + (long long)plane * N * N;
        for (int idx = threadIdx.x; idx < N * L; idx += kThreads) {
            const int r = idx / L, c = idx % L;
            float2 v = src[(long long)r * N + col0 + c];
            float s = sgn(r);
            if constexpr (MODE == COL_WINV_IFFT_CROP) s *= winv(r, col0 + c, N, a.sob_a, a.sob_hl);
            if constexpr (MODE == COL_P_IFFT_CROP) s *= P[(long long)r * N + col0 + c];
            tile[idx] = cscale(v, s);
        }
    }
    __syncthreads();
    fft_lines<N, L, L, 1, INV1>(tile, tw);

    if constexpr (MODE == COL_PAD_FFT_P2_IFFT) {
        // post-sign of the forward and pre-sign of the inverse cancel
        const float rs2 = a.rs * a.rs;
        for (int idx = threadIdx.x; idx < N * L; idx += kThreads) {
            const int r = idx / L, c = idx % L;
            const float p = P[(long long)r * N + col0 + c];
            tile[idx] = cscale(tile[idx], p * p * rs2);
        }
        __syncthreads();
        fft_lines<N, L, L, 1, true>(tile, tw);
    }

    if constexpr (MODE == COL_WINV_IFFT_CROP || MODE == COL_P_IFFT_CROP || MODE == COL_PAD_FFT_P2_IFFT) {
        float2* dst = a.out + (long long)plane * m * N;
        for (int idx = threadIdx.x; idx < m * L; idx += kThreads) {
            const int ri = idx / L, c = idx % L;
            const int r = ri + lo;
            const float s = (MODE == COL_PAD_FFT_P2_IFFT) ? sgn(r) : sgn(r) * a.rs;
            dst[(long long)ri * N + col0 + c] = cscale(tile[r * L + c], s);
        }
    } else {
        const long long pbase = (long long)plane * N * N;
        const float s1 = a.s1 ? a.s1[f] : a.c1;
        const float s2 = a.s2 ? a.s2[f] : a.c2;
        for (int idx = threadIdx.x; idx < N * L; idx += kThreads) {
            const int r = idx / L, c = idx % L;
            const long long o = (long long)r * N + col0 + c;
            float2 v = cscale(tile[idx], sgn(r) * a.rs);
            if constexpr (MODE == COL_PAD_FFT_P) {
                a.out[pbase + o] = cscale(v, P[o]);
            } else if constexpr (MODE == COL_PAD_FFT_P_RESID) {
                const float2 y = a.add1[pbase + o];
                const float p = P[o];
                a.out[pbase + o] = make_float2(s1 * y.x - p * v.x, s1 * y.y - p * v.y);
            } else if constexpr (MODE == COL_PAD_FFT_WINV_ADD) {
                v = cscale(v, winv(r, col0 + c, N, a.sob_a, a.sob_hl));
                if (a.add1) { const float2 u = a.add1[pbase + o]; v.x += s1 * u.x; v.y += s1 * u.y; }
                if (a.add2) { const float2 u = a.add2[pbase + o]; v.x += s2 * u.x; v.y += s2 * u.y; }
                a.out[pbase + o] = v;
            } else if constexpr (MODE == COL_PAD_FFT_GPROD) {
                const float2 g = a.add1[pbase + o];
                reinterpret_cast<float*>(a.out)[pbase + o] = g.x * v.x + g.y * v.y;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// row passes: a workgroup transforms L lines; line = (plane, Omega row i)
// ---------------------------------------------------------------------------

enum RowMode : int {
    ROW_CACHE = 0,   // c = crop_cols(IDFT_1(T))
    ROW_FWD = 1,     // T = DFT_1(pad_cols(rho . c))
    ROW_DERIV = 2,   // dc = crop_cols(IDFT_1(T)); T = DFT_1(pad_cols(drho . c + rho . dc))
    ROW_ADJ = 3,     // u = crop_cols(IDFT_1(T)); aux = conj(c) . u; T = DFT_1(pad_cols(conj(rho) . u))
};

struct RowArgs {
    const float2* in;        // T [planes][m][n]
    float2* out;             // T (may equal in)
    const float2* c;         // [planes][m][m]
    float2* c_out;           // ROW_CACHE output
    const float2* rho;       // [frames][m][m]
    const float2* drho;      // [frames][m][m]
    float2* aux;             // [planes][m][m]
    const int* plane_frame;
    int nlines;              // planes * m
    int m, lo;
    float rs;
    const float2* tw;
};

template <int N, int L, int MODE>
__global__ __launch_bounds__(kThreads) void k_row(RowArgs a) {
    __shared__ float2 tile[L * N];
    __shared__ float2 tw[N];
    const int line0 = blockIdx.x * L;
    const int m = a.m, lo = a.lo;
    for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = a.tw[i];

    if constexpr (MODE == ROW_FWD) {
        for (int idx = threadIdx.x; idx < L * N; idx += kThreads) {
            const int l = idx / N, pos = idx % N;
            const int line = line0 + l;
            float2 v = make_float2(0.f, 0.f);
            const int q = pos - lo;
            if (line < a.nlines && q >= 0 && q < m) {
                const int plane = line / m, i = line % m;
                const int f = a.plane_frame ? a.plane_frame[plane] : 0;
                const float2 cv = a.c[((long long)plane * m + i) * m + q];
                const float2 rv = a.rho[((long long)f * m + i) * m + q];
                v = cscale(cmul(rv, cv), sgn(pos));
            }
            tile[idx] = v;
        }
        __syncthreads();
    } else {
        for (int idx = threadIdx.x; idx < L * N; idx += kThreads) {
            const int l = idx / N, pos = idx % N;
            const int line = line0 + l;
            float2 v = make_float2(0.f, 0.f);
            if (line < a.nlines) v = cscale(a.in[(long long)line * N + pos], sgn(pos));
            tile[idx] = v;
        }
        __syncthreads();
        fft_lines<N, L, 1, N, true>(tile, tw);
        // crop to Omega columns, pointwise products, zero-pad
        for (int idx = threadIdx.x; idx < L * N; idx += kThreads) {
            const int l = idx / N, pos = idx % N;
            const int line = line0 + l;
            const int q = pos - lo;
            float2 z = make_float2(0.f, 0.f);
            if (line < a.nlines && q >= 0 && q < m) {
                const int plane = line / m, i = line % m;
                const float2 u = cscale(tile[idx], sgn(pos) * a.rs);
                const long long oc = ((long long)plane * m + i) * m + q;
                if constexpr (MODE == ROW_CACHE) {
                    a.c_out[oc] = u;
                } else {
                    const int f = a.plane_frame ? a.plane_frame[plane] : 0;
                    const long long orh = ((long long)f * m + i) * m + q;
                    const float2 cv = a.c[oc];
                    const float2 rv = a.rho[orh];
                    if constexpr (MODE == ROW_DERIV) {
                        const float2 dr = a.drho[orh];
                        z = cadd(cmul(dr, cv), cmul(rv, u));
                    } else {  // ROW_ADJ
                        a.aux[oc] = cconjmul(cv, u);
                        z = cconjmul(rv, u);
                    }
                    z = cscale(z, sgn(pos));
                }
            }
            if constexpr (MODE != ROW_CACHE) tile[idx] = z;
        }
        if constexpr (MODE == ROW_CACHE) return;
        __syncthreads();
    }
    fft_lines<N, L, 1, N, false>(tile, tw);
    for (int idx = threadIdx.x; idx < L * N; idx += kThreads) {
        const int l = idx / N, pos = idx % N;
        const int line = line0 + l;
        if (line < a.nlines) a.out[(long long)line * N + pos] = cscale(tile[idx], sgn(pos) * a.rs);
    }
}

}  // namespace nlinv

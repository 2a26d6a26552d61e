// Batched 1D complex FFTs of compile-time length N = 2^p 3^q on lines held in
// LDS, for gfx950 (64-wide wavefronts, 256-thread workgroups).
//
// Algorithm: Stockham auto-sort, radix 8 / 4 / 2 / 3 stages (largest first),
// after Govindaraju et al., "High performance discrete Fourier transforms on
// graphics processors" (SC 2008).  Stage s with radix R and running stride Ns
// takes butterfly j's inputs at j + k N/R, multiplies input k by
// exp(-+2 pi i (j mod Ns) k / (Ns R)), does an R-point DFT in registers and
// writes output k to (j / Ns) Ns R + (j mod Ns) + k Ns.  The output ends in
// natural order.
//
// The butterflies of all lines of a workgroup are flattened over its 256
// threads; each stage reads its inputs into registers, waits at a barrier,
// and writes in place, so one LDS buffer of lines suffices.  Element (line,
// pos) lives at buf[pos * PS + line * LS]: row tiles use PS = 1 (a line is
// contiguous), column tiles PS = lines, LS = 1 (a line is a tile column, so
// consecutive threads touch consecutive lines and consecutive banks).
// Twiddles exp(-2 pi i m / N) come from a table staged in LDS.
#pragma once
#include <hip/hip_runtime.h>

namespace nlinv {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

constexpr int radix_at(int n, int s) {
    int rem = n;
    for (int i = 0;; ++i) {
        if (rem == 1) return 1;
        int r = (rem % 8 == 0) ? 8 : (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3 : rem;
        if (i == s) return r;
        rem /= r;
    }
}

constexpr bool supported_len(int n) {
    if (n < 8 || n > 1024) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// ---- R-point DFTs in registers (sign -1 forward, +1 inverse, unscaled) ----

template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
    // w = exp(-+2 pi i / 3) = -1/2 -+ i sqrt(3)/2
    const float s3 = 0.86602540378443864676f;
    float2 a = v[0], b = v[1], c = v[2];
    float2 t = cadd(b, c);
    float2 d = csub(b, c);
    float2 m = make_float2(a.x - 0.5f * t.x, a.y - 0.5f * t.y);
    // -+ i sqrt(3)/2 (b - c)
    float2 r = INV ? make_float2(-s3 * d.y, s3 * d.x) : make_float2(s3 * d.y, -s3 * d.x);
    v[0] = cadd(a, t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
    float2 a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    float2 s13 = cadd(a1, a3), d13 = mul_mi<INV>(csub(a1, a3));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
    const float h = 0.70710678118654752440f;
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // o[k] *= exp(-+2 pi i k / 8)
    float2 o1 = INV ? make_float2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                    : make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    float2 o2 = mul_mi<INV>(o[2]);
    float2 o3 = INV ? make_float2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                    : make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dftR(float2* v) {
    if constexpr (R == 2) dft2<INV>(v);
    else if constexpr (R == 3) dft3<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else if constexpr (R == 8) dft8<INV>(v);
}

// ---- one Stockham stage and the stage chain -------------------------------

template <int N, int NL, int PS, int LS, bool INV, int S, int NS>
struct FFTStage {
    static __device__ __forceinline__ void run(float2* buf, const float2* tw) {
        constexpr int R = radix_at(N, S);
        if constexpr (R > 1) {
            constexpr int B = N / R;                 // butterflies per line
            constexpr int TOT = B * NL;              // butterflies per workgroup
            constexpr int PER = (TOT + kThreads - 1) / kThreads;
            constexpr int TWS = N / (NS * R);
            float2 v[PER][R];
            int jj[PER], ll[PER];
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const int g = threadIdx.x + it * kThreads;
                jj[it] = -1;
                if (TOT % kThreads == 0 || g < TOT) {
                    int j, l;
                    if constexpr (PS == 1) { j = g % B; l = g / B; }
                    else { l = g % NL; j = g / NL; }
                    jj[it] = j;
                    ll[it] = l;
                    const int tstep = (j % NS) * TWS;
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        float2 a = buf[(j + k * B) * PS + l * LS];
                        if (NS > 1 && k > 0) {
                            const float2 w = tw[k * tstep];
                            a = INV ? cmulc(a, w) : cmul(a, w);
                        }
                        v[it][k] = a;
                    }
                    dftR<R, INV>(v[it]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const int j = jj[it];
                if (j >= 0) {
                    const int l = ll[it];
                    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
                    for (int k = 0; k < R; ++k) buf[(base + k * NS) * PS + l * LS] = v[it][k];
                }
            }
            __syncthreads();
            FFTStage<N, NL, PS, LS, INV, S + 1, NS * R>::run(buf, tw);
        }
    }
};

// Transform all NL lines in `buf` (unscaled; forward = exp(-2 pi i k r / N)).
// Callers must have completed their writes to buf and tw with a barrier.
template <int N, int NL, int PS, int LS, bool INV>
__device__ __forceinline__ void fft_lines(float2* buf, const float2* tw) {
    FFTStage<N, NL, PS, LS, INV, 0, 1>::run(buf, tw);
}

}  // namespace nlinv

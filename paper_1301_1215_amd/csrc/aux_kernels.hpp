// Coil-sum, image, CG vector and FP64 reduction kernels (not size-templated;
// built once, in the host library's translation unit).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_scalars.hpp"
#include "fft_core.hpp"

namespace nlinv {

// ---------------------------------------------------------------------------
// coil sums over the planes of each frame (fixed order: deterministic)
// ---------------------------------------------------------------------------

// out[f][e] = sum_{p in f} aux[p][e] + s1_f add1[f][e] + s2_f add2[f][e]
// One thread per Omega pixel, one workgroup per (frame, segment of
// `seg_len` pixels); with `partial` set it also writes Re<add1, out> of its
// segment to partial[poff + f*segs + k].
// With self_dot the partial is |out|^2 instead.
// CG form (r_upd set): the sum q (with add1 = p, s1 = alpha) is not stored;
// instead r -= a_f q and dx += a_f p, and the partial is |r|^2.
struct CoilSumArgs {
    const float2* aux;       // [planes][E]
    float2* out;             // [frames][E]
    const float2* add1;
    const float2* add2;
    const float* s1;
    const float* s2;
    float c1, c2;
    const int* frame_plane0; // nullable: single frame with `nplanes` planes
    const int* frame_planes;
    int nplanes;
    int nframes;
    int E;                   // elements per frame (m*m)
    int segs, seg_len;       // seg_len <= kThreads
    double* partial;
    long long poff;
    int self_dot;
    float2* r_upd;           // CG form: rho part of r (in place), nullable
    float2* dx_upd;          // rho part of dx (in place)
    const float* cg_a;       // [frames] CG step a
};

__global__ __launch_bounds__(kThreads) void k_coil_sum(CoilSumArgs a) {
    __shared__ double red[4];
    const int f = blockIdx.x / a.segs, k = blockIdx.x % a.segs;
    const int e = k * a.seg_len + threadIdx.x;
    const int p0 = a.frame_plane0 ? a.frame_plane0[f] : 0;
    const int np = a.frame_planes ? a.frame_planes[f] : a.nplanes;
    double acc = 0.0;
    if (threadIdx.x < a.seg_len && e < a.E) {
        const long long g = (long long)f * a.E + e;
        const float2* src = a.aux + (long long)p0 * a.E + e;
        // the pointwise operands first, so their loads overlap the plane loads
        const float c1 = a.s1 ? a.s1[f] : a.c1;
        const float c2 = a.s2 ? a.s2[f] : a.c2;
        const float2 zero = make_float2(0.f, 0.f);
        const float2 u1 = a.add1 ? a.add1[g] : zero;
        const float2 u2 = a.add2 ? a.add2[g] : zero;
        float2 r = a.r_upd ? a.r_upd[g] : zero;
        float2 d = a.r_upd ? a.dx_upd[g] : zero;
        // four independent chains over the planes (four loads in flight),
        // combined in a fixed order
        float2 s0 = zero, s1 = zero, s2 = zero, s3 = zero;
        int p = 0;
        for (; p + 3 < np; p += 4) {
            const float2 v0 = src[(long long)p * a.E], v1 = src[(long long)(p + 1) * a.E];
            const float2 v2 = src[(long long)(p + 2) * a.E], v3 = src[(long long)(p + 3) * a.E];
            s0 = cadd(s0, v0);
            s1 = cadd(s1, v1);
            s2 = cadd(s2, v2);
            s3 = cadd(s3, v3);
        }
        if (p < np) s0 = cadd(s0, src[(long long)p * a.E]);
        if (p + 1 < np) s1 = cadd(s1, src[(long long)(p + 1) * a.E]);
        if (p + 2 < np) s2 = cadd(s2, src[(long long)(p + 2) * a.E]);
        float2 s = cadd(cadd(s0, s1), cadd(s2, s3));
        s.x += c1 * u1.x + c2 * u2.x;
        s.y += c1 * u1.y + c2 * u2.y;
        if (a.r_upd) {
            const float av = a.cg_a[f];
            r.x -= av * s.x;
            r.y -= av * s.y;
            a.r_upd[g] = r;
            d.x += av * u1.x;
            d.y += av * u1.y;
            a.dx_upd[g] = d;
            acc = (double)(r.x * r.x + r.y * r.y);
        } else {
            a.out[g] = s;
            if (a.self_dot) acc = (double)(s.x * s.x + s.y * s.y);
            else if (a.partial && a.add1) acc = (double)(u1.x * s.x + u1.y * s.y);
        }
    }
    if (a.partial) {
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) a.partial[a.poff + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_coil_sum_real(const float* gprod, float* out, int nplanes, int E) {
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < E; e += gridDim.x * kThreads) {
        float s = 0.f;
        for (int p = 0; p < nplanes; ++p) s += gprod[(long long)p * E + e];
        out[e] = s;
    }
}

// image[f][e] = rho[f][e] . sqrt(sum_{p in f} |c[p][e]|^2) * inv_s[f]
__global__ __launch_bounds__(kThreads) void k_image(const float2* rho, const float2* c, float2* img,
                                                    const int* frame_plane0, const int* frame_planes,
                                                    int nplanes, int nframes, int E, const float* inv_s) {
    const long long tot = (long long)nframes * E;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const int f = (int)(g / E), e = (int)(g % E);
        const int p0 = frame_plane0 ? frame_plane0[f] : 0;
        const int np = frame_planes ? frame_planes[f] : nplanes;
        float s = 0.f;
        for (int p = 0; p < np; ++p) {
            const float2 v = c[(long long)(p0 + p) * E + e];
            s += v.x * v.x + v.y * v.y;
        }
        const float sc = sqrtf(s) * (inv_s ? inv_s[f] : 1.0f);
        img[g] = cscale(rho[g], sc);
    }
}

// ---------------------------------------------------------------------------
// CG vector kernels: one workgroup per segment of the class-wide vector
// ---------------------------------------------------------------------------

struct VecPtrs {
    float2* c0; float2* c1;   // chat parts
    float2* r0; float2* r1;   // rho parts
};

enum VecOp : int {
    VEC_DOT = 0,        // partial = Re<v0, v1>
    VEC_ADD = 1,        // v0 += v1
};

template <int OP>
__global__ __launch_bounds__(kThreads) void k_vec(SegGeom g, VecPtrs v, double* partial) {
    __shared__ double red[4];
    bool is_c; int owner, f, len; long long base;
    seg_locate(g, blockIdx.x, is_c, owner, f, base, len);
    float2* x0 = is_c ? v.c0 : v.r0;
    float2* x1 = is_c ? v.c1 : v.r1;
    float4* y0 = reinterpret_cast<float4*>(x0 + base);
    float4* y1 = reinterpret_cast<float4*>(x1 + base);
    const int n4 = len / 2;
    double acc = 0.0;
    (void)f; (void)owner;
    for (int i = threadIdx.x; i < n4; i += kThreads) {
        if constexpr (OP == VEC_DOT) {
            const float4 p = y0[i], q = y1[i];
            acc += (double)p.x * q.x + (double)p.y * q.y + (double)p.z * q.z + (double)p.w * q.w;
        } else if constexpr (OP == VEC_ADD) {
            float4 p = y0[i];
            const float4 r = y1[i];
            p.x += r.x; p.y += r.y; p.z += r.z; p.w += r.w;
            y0[i] = p;
        }
    }
    if constexpr (OP == VEC_DOT) {
        const double t = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// One workgroup per frame: total of its partials, then the scalar step.
// One wavefront per frame: the frame's scalars and its partials are loaded
// together, summed in a fixed order, then the scalar step.
__global__ __launch_bounds__(64) void k_scalar(ScalarStep ss, Scalars sc) {
    fold_scalar_step(ss, sc);
}

// per-frame: alpha[f] = value, alpha[F + f] = -value
__global__ void k_set_alpha(float* alpha, int nframes, float value) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nframes) { alpha[f] = value; alpha[nframes + f] = -value; }
}

// x[f][e] = s_f * src[f][e] (src nullable -> s_f * 1) on rho parts
__global__ __launch_bounds__(kThreads) void k_scale_rho(float2* x, const float2* src, const float* s,
                                                        int nframes, int E, int use_inv) {
    const long long tot = (long long)nframes * E;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const int f = (int)(g / E);
        const float sf = s[f];
        const float2 v = src ? src[g] : make_float2(1.f, 0.f);
        x[g] = cscale(v, sf);
        (void)use_inv;
    }
}

// Convert planes between row-major [planes][n][n] and the column-tiled
// layout [planes][n/tw][n][tw] used inside a solve (to_tiled = 0: back).
template <class T>
__global__ __launch_bounds__(kThreads) void k_tile(const T* src, T* dst, int nplanes, int n, int tw,
                                                  int to_tiled) {
    const long long nn = (long long)n * n, tot = nplanes * nn;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const long long pl = g / nn, e = g % nn;
        const int r = (int)(e / n), c = (int)(e % n);
        const long long t = pl * nn + ((long long)(c / tw) * n + r) * tw + (c % tw);
        if (to_tiled) dst[t] = src[g];
        else dst[g] = src[t];
    }
}

// Bandwidth probe: a plain 16-byte-per-thread streaming copy (the practical
// HBM ceiling, and the known-size copy that calibrates traffic counters).
__global__ __launch_bounds__(kThreads) void k_stream_copy(const float4* __restrict__ src,
                                                          float4* __restrict__ dst, long long n16) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n16; i += (long long)gridDim.x * kThreads)
        dst[i] = src[i];
}

__global__ __launch_bounds__(kThreads) void k_fill(float2* x, long long n, float2 v) {
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < n;
         g += (long long)gridDim.x * kThreads) x[g] = v;
}

}  // namespace nlinv

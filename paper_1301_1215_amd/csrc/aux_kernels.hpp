// Coil-sum, image, CG vector and FP64 reduction kernels (not size-templated;
// built once, in the host library's translation unit).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_scalars.hpp"
#include "coil_sum.hpp"
#include "fft_core.hpp"

namespace nlinv {

// ---------------------------------------------------------------------------
// coil sums over the planes of each frame (fixed order: deterministic)
// ---------------------------------------------------------------------------

// k_coil_sum: a coil sum on its own (one 256-thread workgroup per segment)
__global__ __launch_bounds__(kThreads) void k_coil_sum(CoilSumArgs a) {
    __shared__ double red[kThreads / 64];
    coil_sum_block<kThreads>(a, blockIdx.x, red);
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

// The same conversion for up to kTileBatch frames in one launch: entry
// blockIdx.y copies np[y] planes from src[y] to dst[y].
constexpr int kTileBatch = 16;
template <class T>
struct TileBatch {
    const T* src[kTileBatch];
    T* dst[kTileBatch];
    int np[kTileBatch];
};
template <class T>
__global__ __launch_bounds__(kThreads) void k_tile_batch(TileBatch<T> b, int n, int tw, int to_tiled) {
    const T* src = b.src[blockIdx.y];
    T* dst = b.dst[blockIdx.y];
    const long long nn = (long long)n * n, tot = b.np[blockIdx.y] * nn;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const long long pl = g / nn, e = g % nn;
        const int r = (int)(e / n), c = (int)(e % n);
        const long long t = pl * nn + ((long long)(c / tw) * n + r) * tw + (c % tw);
        if (to_tiled) dst[t] = src[g];
        else dst[g] = src[t];
    }
}

// Up to kCopyBatch device-to-device copies of 8-byte words in one launch:
// entry blockIdx.y copies n[y] words from src[y] to dst[y].
constexpr int kCopyBatch = 48;
struct CopyBatch {
    const uint64_t* src[kCopyBatch];
    uint64_t* dst[kCopyBatch];
    long long n[kCopyBatch];
};
__global__ __launch_bounds__(kThreads) void k_copy_batch(CopyBatch b) {
    const uint64_t* src = b.src[blockIdx.y];
    uint64_t* dst = b.dst[blockIdx.y];
    const long long n = b.n[blockIdx.y];
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// the band of the sensitivities a solve keeps (rows and columns
// [klo, klo + kb) of k-space), against the caller's whole [n][n] planes
// ---------------------------------------------------------------------------

// Up to kTileBatch frames per launch; entry blockIdx.y covers np[y] planes.
struct BandBatch {
    const float2* src[kTileBatch];   // k_band_in: caller planes [np][n][n]
    const float2* band[kTileBatch];  // k_chat_out: band planes (solve layout)
    float2* dst[kTileBatch];         // k_band_in: band planes; k_chat_out: caller planes
    const float2* x0[kTileBatch];    // k_chat_out / k_inert_dist: the start x0 (nullable: 0)
    const float2* ref[kTileBatch];   // the caller's x_ref (nullable: x_ref = x0)
    int np[kTileBatch];
    int plane0[kTileBatch];          // k_inert_dist: class plane of the entry's first plane
    int frame[kTileBatch];           // k_chat_out: class frame of the entry
};

// band of caller planes -> solve layout [kb/tw][kb][tw] per plane
__global__ __launch_bounds__(kThreads) void k_band_in(BandBatch b, int n, int klo, int kb, int tw) {
    const float2* src = b.src[blockIdx.y];
    float2* dst = b.dst[blockIdx.y];
    const long long kk = (long long)kb * kb, tot = b.np[blockIdx.y] * kk;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const long long pl = g / kk, e = g % kk;
        const int r = (int)(e / kb), c = (int)(e % kb);
        dst[pl * kk + ((long long)(c / tw) * kb + r) * tw + (c % tw)] =
            src[pl * (long long)n * n + (long long)(klo + r) * n + klo + c];
    }
}

// The caller's planes of the result: the band from the solve layout, the
// rest x_ref + theta (x0 - x_ref) (x_ref = x0 when ref is null, x0 = 0 when
// x0 is null); theta = inert[frame][1].  x0 or ref may alias dst (each
// element is read before it is written, by the same thread).
__global__ __launch_bounds__(kThreads) void k_chat_out(BandBatch b, const double* inert, int n, int klo, int kb,
                                                      int tw) {
    const float2* band = b.band[blockIdx.y];
    const float2* x0 = b.x0[blockIdx.y];
    const float2* ref = b.ref[blockIdx.y];
    float2* dst = b.dst[blockIdx.y];
    const float th = (float)inert[(long long)b.frame[blockIdx.y] * kInertLen + 1];
    const long long nn = (long long)n * n, kk = (long long)kb * kb, tot = b.np[blockIdx.y] * nn;
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < tot;
         g += (long long)gridDim.x * kThreads) {
        const long long pl = g / nn, e = g % nn;
        const int r = (int)(e / n) - klo, c = (int)(e % n) - klo;
        float2 v;
        if ((unsigned)r < (unsigned)kb && (unsigned)c < (unsigned)kb) {
            v = band[pl * kk + ((long long)(c / tw) * kb + r) * tw + (c % tw)];
        } else {
            const float2 x = x0 ? x0[g] : make_float2(0.f, 0.f);
            if (ref) {
                const float2 q = ref[g];
                v = make_float2(q.x + th * (x.x - q.x), q.y + th * (x.y - q.y));
            } else {
                v = x;
            }
        }
        dst[g] = v;
    }
}

// partial[(plane0 + p) * segs + g] = |x0 - ref|^2 over rows g*rows..(g+1)*rows
// of plane p, outside the band (x0 null: 0; ref null: 0), in FP64; one
// workgroup per (plane, row segment), a fixed order
__global__ __launch_bounds__(kThreads) void k_inert_dist(BandBatch b, double* partial, int n, int klo, int kb,
                                                        int segs) {
    __shared__ double red[kThreads / 64];
    const int y = blockIdx.y, pl = blockIdx.x / segs, g = blockIdx.x % segs;
    if (pl >= b.np[y]) return;
    const float2* x0 = b.x0[y];
    const float2* ref = b.ref[y];
    const long long base = (long long)pl * n * n;
    const int rows = (n + segs - 1) / segs, r0 = g * rows, r1 = min(n, r0 + rows);
    double acc = 0.0;
    if (ref) {
        for (int r = r0; r < r1; ++r) {
            const bool rin = (unsigned)(r - klo) < (unsigned)kb;
            for (int c = threadIdx.x; c < n; c += kThreads) {
                if (rin && (unsigned)(c - klo) < (unsigned)kb) continue;
                const long long e = base + (long long)r * n + c;
                const float2 x = x0 ? x0[e] : make_float2(0.f, 0.f);
                const float2 q = ref[e];
                const double dx = (double)x.x - q.x, dy = (double)x.y - q.y;
                acc += dx * dx + dy * dy;
            }
        }
    }
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(long long)(b.plane0[y] + pl) * segs + g] = t;
}

// Start of a solve: the record of the components outside the band for every
// frame of a class (D from the per-plane partials, `segs` per plane, in
// order, or 0 when partial is null; theta = 1)
__global__ __launch_bounds__(kThreads) void k_inert_init(double* inert, const double* partial, int segs,
                                                        const int* frame_plane0, const int* frame_planes,
                                                        int nplanes, int nframes) {
    for (int f = blockIdx.x * kThreads + threadIdx.x; f < nframes; f += gridDim.x * kThreads) {
        double d = 0.0;
        if (partial) {
            const int p0 = frame_plane0 ? frame_plane0[f] : 0;
            const int np = frame_planes ? frame_planes[f] : nplanes;
            for (long long i = (long long)p0 * segs; i < (long long)(p0 + np) * segs; ++i) d += partial[i];
        }
        double* in = inert + (long long)f * kInertLen;
        in[0] = d;
        in[1] = 1.0;
        for (int k = 2; k < kInertLen; ++k) in[k] = 0.0;
    }
}

// Bandwidth probe: a streaming copy (the practical HBM ceiling, and the
// known-size copy that calibrates traffic counters).  Each thread moves
// kProbeUnroll 16-byte words per round, all loads issued before the stores
// (one wavefront keeps 4 KiB in flight), with non-temporal hints: the data
// are touched once.
constexpr int kProbeUnroll = 4;
typedef float probe_v4 __attribute__((ext_vector_type(4)));   // a native 16-byte vector
__global__ __launch_bounds__(kThreads) void k_stream_copy(const probe_v4* __restrict__ src,
                                                          probe_v4* __restrict__ dst, long long n16) {
    const long long step = (long long)gridDim.x * kThreads * kProbeUnroll;
    for (long long b = (long long)blockIdx.x * kThreads * kProbeUnroll + threadIdx.x; b < n16; b += step) {
        probe_v4 v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const long long i = b + (long long)u * kThreads;
            if (i < n16) v[u] = __builtin_nontemporal_load(src + i);
        }
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const long long i = b + (long long)u * kThreads;
            if (i < n16) __builtin_nontemporal_store(v[u], dst + i);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_fill(float2* x, long long n, float2 v) {
    for (long long g = (long long)blockIdx.x * kThreads + threadIdx.x; g < n;
         g += (long long)gridDim.x * kThreads) x[g] = v;
}

}  // namespace nlinv

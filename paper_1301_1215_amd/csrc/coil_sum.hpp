// Coil sums over the planes of each frame (fixed order: deterministic),
// as a workgroup body: a kernel of their own (k_coil_sum) or extra
// workgroups of the CG-update column pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_scalars.hpp"
#include "fft_core.hpp"

namespace nlinv {

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
    int segs, seg_len;       // seg_len <= the workgroup size
    double* partial;
    long long poff;
    int self_dot;
    float2* r_upd;           // CG form: rho part of r (in place), nullable
    float2* dx_upd;          // rho part of dx (in place)
    int dx_zero;             // dx starts from 0 (first CG iteration): not read
    const float* cg_a;       // [frames] CG step a
    int group;               // > 1: aux holds sums over groups of that many coils,
                             // [planes / group][E] (frames' plane ranges divisible by it)
};

// One (frame, segment) of the sum with NT threads (seg_len <= NT); `red`
// holds NT/64 doubles.
template <int NT>
__device__ __forceinline__ void coil_sum_block(const CoilSumArgs& a, int b, double* red) {
    const int f = b / a.segs, k = b % a.segs;
    const int e = k * a.seg_len + threadIdx.x;
    const int gs = a.group > 1 ? a.group : 1;
    const int p0 = (a.frame_plane0 ? a.frame_plane0[f] : 0) / gs;
    const int np = (a.frame_planes ? a.frame_planes[f] : a.nplanes) / gs;
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
        float2 d = (a.r_upd && !a.dx_zero) ? a.dx_upd[g] : zero;
        // The sum's order depends on the frame alone (not on the batch or on
        // which pass formed the partial sums): a frame whose coil count is a
        // multiple of 4 sums each group of 4 consecutive coils as
        // (c0 + c2) + (c1 + c3) (what the adjoint row pass forms when it
        // groups coils), then the groups; otherwise the coils.  The items
        // are summed in eight independent chains (eight loads in flight),
        // combined in a fixed order.
        const bool quads = gs == 4 || np % 4 == 0;
        const int nitems = gs == 4 ? np : (quads ? np / 4 : np);
        auto item = [&](int i) -> float2 {
            if (gs == 4 || !quads) return src[(long long)i * a.E];
            const float2* q = src + (long long)4 * i * a.E;
            return cadd(cadd(q[0], q[2 * (long long)a.E]), cadd(q[a.E], q[3 * (long long)a.E]));
        };
        constexpr int U = 8;
        float2 sc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sc[u] = zero;
        int i0 = 0;
        for (; i0 + U - 1 < nitems; i0 += U) {
            float2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = item(i0 + u);
#pragma unroll
            for (int u = 0; u < U; ++u) sc[u] = cadd(sc[u], v[u]);
        }
#pragma unroll
        for (int u = 0; u < U - 1; ++u)
            if (i0 + u < nitems) sc[u] = cadd(sc[u], item(i0 + u));
        float2 s = cadd(cadd(cadd(sc[0], sc[1]), cadd(sc[2], sc[3])), cadd(cadd(sc[4], sc[5]), cadd(sc[6], sc[7])));
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
        const double t = wg_sum<NT>(acc, red);
        if (threadIdx.x == 0) a.partial[a.poff + b] = t;
    }
}

}  // namespace nlinv

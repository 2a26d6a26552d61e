// Per-frame CG and Newton scalars: FP64 partial-sum geometry, fixed-order
// frame totals and the scalar step logic, shared by the vector kernels and
// the pass kernels that fold a scalar step into their launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace nlinv {

// ---------------------------------------------------------------------------
// segment geometry of a class-wide CG vector:
//   chat part [planes][n*n] in `cseg` segments per plane,
//   rho part  [frames][m*m] in `rseg` segments per frame;
// one FP64 partial per segment, summed per frame in a fixed order.
// ---------------------------------------------------------------------------

struct SegGeom {
    int nplanes, nframes;
    int cn, rn;          // elements per plane / per frame (complex)
    int cseg, rseg;      // segments per plane / per frame
    int clen, rlen;      // elements per segment (even), last one ragged
    const int* plane_frame;
};

__device__ __forceinline__ void seg_locate(const SegGeom& g, int s, bool& is_c, int& owner, int& f,
                                           long long& base, int& len) {
    const int ncs = g.nplanes * g.cseg;
    if (s < ncs) {
        is_c = true;
        owner = s / g.cseg;
        const int k = s % g.cseg;
        f = g.plane_frame ? g.plane_frame[owner] : 0;
        base = (long long)owner * g.cn + (long long)k * g.clen;
        len = min(g.clen, g.cn - k * g.clen);
    } else {
        is_c = false;
        const int t = s - ncs;
        owner = t / g.rseg;
        const int k = t % g.rseg;
        f = owner;
        base = (long long)owner * g.rn + (long long)k * g.rlen;
        len = min(g.rlen, g.rn - k * g.rlen);
    }
}

// Sum over a 256-thread workgroup in a fixed order (wavefront shuffle, then
// the 4 waves); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// Sum over an NT-thread workgroup in a fixed order (wavefront shuffle, then
// the waves in order); the result is valid in thread 0 and `red` (NT/64
// doubles) is free again on return.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Sensitivity components outside the band of k-space that the solve keeps
// (where 1/w is below 2^-40) do not reach DF in single precision: there the
// normal operator is alpha I, and CG moves them along a fixed direction.
// With e = x_n - x_ref on those components and b = -alpha e, every CG vector
// there is a real multiple of b: r = rho_k b, p = pi_k b, dx = xi_k b, with
// rho_0 = pi_0 = 1, xi_0 = 0 and, for the step a_k and direction weight
// beta_k of the whole vector,
//   rho_{k+1} = rho_k - a_k alpha pi_k,   xi_{k+1} = xi_k + a_k pi_k,
//   pi_{k+1} = rho_{k+1} + beta_{k+1} pi_k;
// they add rho_k^2 |b|^2 to <r, r> and alpha pi_k^2 |b|^2 to Re<p, N p>, and
// after the Newton step e <- (1 - alpha xi_K) e.  So only |e_0|^2 = D (set
// when the solve starts) and theta (e_n = theta e_0) are kept per frame; the
// components themselves are written once, at the end: x_ref + theta e_0.
// Per-frame record: [0] D, [1] theta, [2] |b|^2 of the current Newton step,
// then (rho, pi, xi) in two slots by the parity of the CG iteration (a step
// folded into a pass reads one slot while its first workgroup writes the
// other).
constexpr int kInertLen = 9;

// CG and Newton scalars of every frame of a class, all on the device.
struct Scalars {
    double* rr;        // [2][F] <r, r>, by the parity of the CG iteration it belongs to
                       // (a step folded into a pass reads one while it writes the other)
    float* a;          // [F] CG step a = rr / gamma
    float* beta;       // [F]
    int* brk;          // [F] breakdown in the current Newton step
    float* s;          // [F] data scale
    float* inv_s;      // [F]
    double* stats;     // [F][stats_len]
    double* inert;     // [F][kInertLen]: the components outside the band (see above)
    int stats_len;
    int nframes;       // F
};

enum ScalarOp : int {
    SC_NONE = -1,
    SC_YNORM = 0,      // s = scale_norm / ||y|| (scale_norm > 0 and ||y|| > 0), else 1
    SC_R0NORM = 1,     // stats[2 + step] = ||r0||
    SC_RR0 = 2,        // rr (of CG iteration 0) = <b, b>; new Newton step: clear breakdown
    SC_GAMMA = 3,      // gamma = Re<p, q> (or |DF p|^2 + alpha |p|^2); a = rr / gamma or breakdown
    SC_RR = 4,         // after CG iteration `it`: rr' = <r, r>; beta = rr'/rr; rr of
                       // iteration it+1 = rr'; stats of iteration `it`
};

// Where a scalar op is applied: which op, geometry of its partials, indices
// for the stats.  With `partial2` set the total is
// sum(partial) + alpha * sum(partial2) (geometry g2).  alpha is the Newton
// step's regularisation weight (the same for every frame of a solve); SC_RR0,
// SC_GAMMA and SC_RR use it for the components outside the band.
struct ScalarStep {
    int op;
    SegGeom g;
    const double* partial;
    SegGeom g2;
    const double* partial2;
    float alpha;
    const int* frame_plane0;
    const int* frame_planes;
    float scale_norm;
    int step, it, nsteps, ncg;
};

// The frame's scalars the step logic reads, loaded before the partials are
// summed so that the two memory round trips overlap.
struct FrameScalars {
    double rr, flags;
    int brk;
    float a;                     // the CG step of this iteration (0 after a breakdown)
    double B2, irho, ipi, ixi;   // components outside the band: |b|^2 and this iteration's slot
};
// <r, r> of CG iteration `it` of frame f
__device__ __forceinline__ double* rr_of(const Scalars& sc, int it, int f) {
    return sc.rr + (long long)(it & 1) * sc.nframes + f;
}
// slot of (rho, pi, xi) at the start of CG iteration `it`
__device__ __forceinline__ double* inert_slot(const Scalars& sc, int f, int it) {
    return sc.inert + (long long)f * kInertLen + 3 + 3 * (it & 1);
}
__device__ __forceinline__ FrameScalars load_frame_scalars(const ScalarStep& ss, const Scalars& sc, int f) {
    const int it = ss.op == SC_RR0 ? 0 : ss.it;
    const double* in = sc.inert + (long long)f * kInertLen;
    const double* sl = inert_slot(sc, f, it);
    return FrameScalars{*rr_of(sc, it, f), sc.stats[(long long)f * sc.stats_len + 1], sc.brk[f], sc.a[f],
                        in[2], sl[0], sl[1], sl[2]};
}

// After CG iteration ss.it: the coefficients of r and dx outside the band,
// and the total <r, r> with their share added to t (the band's total).
__device__ __forceinline__ double rr_after(const ScalarStep& ss, const FrameScalars& fs, double t, double& rho1,
                                           double& xi1) {
    const double a = (double)fs.a;
    rho1 = fs.irho - a * (double)ss.alpha * fs.ipi;
    xi1 = fs.ixi + a * fs.ipi;
    return t + rho1 * rho1 * fs.B2;
}

// beta of the direction after CG iteration ss.it, from the band's total t of
// <r, r> (SC_RR records the same total)
__device__ __forceinline__ float cg_beta(const ScalarStep& ss, const FrameScalars& fs, double t) {
    double rho1, xi1;
    const double tt = rr_after(ss, fs, t, rho1, xi1);
    return fs.brk ? 0.f : (float)(tt / fs.rr);
}

// The CG step a = rr / gamma after the band's total t of Re<p, N p>, or 0
// on a breakdown (SC_GAMMA records the same value)
__device__ __forceinline__ bool gamma_breaks(const FrameScalars& fs, double g) {
    return fs.brk || fs.rr == 0.0 || !(g > 0.0) || !isfinite(fs.rr);
}
__device__ __forceinline__ double gamma_total(const ScalarStep& ss, const FrameScalars& fs, double t) {
    return t + (double)ss.alpha * fs.ipi * fs.ipi * fs.B2;   // alpha |p|^2 outside the band
}
__device__ __forceinline__ float cg_step(const ScalarStep& ss, const FrameScalars& fs, double t) {
    const double g = gamma_total(ss, fs, t);
    return gamma_breaks(fs, g) ? 0.f : (float)(fs.rr / g);
}

// The scalar logic for frame f given the total t and the frame's scalars
// as loaded before (thread 0 only).
__device__ __forceinline__ void scalar_apply(const ScalarStep& ss, const Scalars& sc, int f, double t,
                                             const FrameScalars& fs) {
    double* st = sc.stats + (long long)f * sc.stats_len;
    const int op = ss.op;
    if (op == SC_YNORM) {
        const double nrm = sqrt(t);
        const float s = (ss.scale_norm > 0.f && nrm > 0.0) ? (float)(ss.scale_norm / nrm) : 1.0f;
        sc.s[f] = s;
        sc.inv_s[f] = 1.0f / s;
        st[0] = (double)s;
        st[1] = 0.0;
        if (!isfinite(nrm)) st[1] = 2.0;
    } else if (op == SC_R0NORM) {
        st[2 + ss.step] = sqrt(t);
        if (!isfinite(t)) st[1] = (double)((int)fs.flags | 2);
    } else if (op == SC_RR0) {
        // b = -alpha e outside the band: |b|^2 = alpha^2 theta^2 D
        double* in = sc.inert + (long long)f * kInertLen;
        const double al = (double)ss.alpha, th = in[1];
        const double B2 = al * al * th * th * in[0];
        in[2] = B2;
        double* sl = inert_slot(sc, f, 0);
        sl[0] = 1.0;
        sl[1] = 1.0;
        sl[2] = 0.0;
        *rr_of(sc, 0, f) = t + B2;
        sc.brk[f] = 0;
    } else if (op == SC_GAMMA) {
        t = gamma_total(ss, fs, t);
        const double rr = fs.rr;
        if (gamma_breaks(fs, t)) {
            if (!fs.brk) {
                int fl = (int)fs.flags | 1;
                if (!isfinite(t) || !isfinite(rr)) fl |= 2;
                st[1] = (double)fl;
            }
            sc.brk[f] = 1;
            sc.a[f] = 0.f;
        } else {
            sc.a[f] = (float)(rr / t);
        }
    } else if (op == SC_RR) {
        double* slot = st + 2 + ss.nsteps + ss.step * ss.ncg + ss.it;
        double rho1, xi1;
        const double tt = rr_after(ss, fs, t, rho1, xi1);
        float beta = 0.f;
        if (fs.brk) {
            *slot = -1.0;
        } else {
            if (!isfinite(tt)) st[1] = (double)((int)fs.flags | 2);
            beta = (float)(tt / fs.rr);
            *rr_of(sc, ss.it + 1, f) = tt;
            *slot = tt;
        }
        sc.beta[f] = beta;
        double* nx = inert_slot(sc, f, ss.it + 1);
        nx[0] = rho1;
        nx[1] = rho1 + (double)beta * fs.ipi;
        nx[2] = xi1;
        if (ss.it == ss.ncg - 1) {   // end of the Newton step: e <- (1 - alpha xi_K) e
            double* in = sc.inert + (long long)f * kInertLen;
            in[1] *= 1.0 - (double)ss.alpha * xi1;
        }
    }
}

// Fixed-order total of frame f computed by one wavefront (lanes 0..63 of
// the calling workgroup, no LDS, no barrier: callable inside a branch that
// only the first wavefront takes); valid in lane 0.
__device__ __forceinline__ double frame_total_wave(const SegGeom& g, const double* partial, int f,
                                                   const int* frame_plane0, const int* frame_planes) {
    const int lane = threadIdx.x & 63;
    const int p0 = frame_plane0 ? frame_plane0[f] : 0;
    const int np = frame_planes ? frame_planes[f] : g.nplanes;
    const int nc = np * g.cseg;
    const int tot = nc + g.rseg;
    const double* cpart = partial + (long long)p0 * g.cseg;
    const double* rpart = partial + (long long)g.nplanes * g.cseg + (long long)f * g.rseg;
    // rounds of U independent loads per lane (latency-bound otherwise),
    // accumulated in a fixed order
    constexpr int U = 8;
    double acc = 0.0;
    for (int base = 0; base < tot; base += 64 * U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * 64 + lane;
            v[u] = i < nc ? cpart[i] : (i < tot ? rpart[i - nc] : 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    return acc;
}

// A scalar step folded into a kernel launch: its first wavefronts compute
// the totals of every frame and apply the step (op == SC_NONE: nothing).
__device__ __forceinline__ void fold_scalar_step(const ScalarStep& ss, const Scalars& sc) {
    if (ss.op == SC_NONE || ss.partial == nullptr || threadIdx.x >= 64) return;
    for (int f = blockIdx.x; f < ss.g.nframes; f += gridDim.x) {
        const FrameScalars fs = load_frame_scalars(ss, sc, f);
        double t = frame_total_wave(ss.g, ss.partial, f, ss.frame_plane0, ss.frame_planes);
        if (ss.partial2) {
            const double t2 = frame_total_wave(ss.g2, ss.partial2, f, ss.frame_plane0, ss.frame_planes);
            if (threadIdx.x == 0) t += (double)ss.alpha * t2;
        }
        if (threadIdx.x == 0) scalar_apply(ss, sc, f, t, fs);
    }
}

}  // namespace nlinv

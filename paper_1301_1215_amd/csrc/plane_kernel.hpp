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

// ---------------------------------------------------------------------------
// A CG iteration of the solve (Eq. 3) on small grids in two launches:
// k_plane_cg (one workgroup per coil plane) folds the previous iteration's
// <r, r> into beta, updates the direction p = r + beta p and applies the
// whole-plane normal operator to it, writing q = W^{-H} E(conj(rho) v) on the
// band, the coil products conj(c) v and the partials of |DF p|^2 and |p|^2;
// k_plane_cg_update then forms the step a = <r, r> / (|DF p|^2 + alpha |p|^2)
// in every workgroup and applies r -= a N p, x += a p (the rho part through
// the coil sum), writing the <r, r> partials the next iteration folds.  The
// scalar logic is the one of the five-pass iteration (cg_scalars.hpp).
// ---------------------------------------------------------------------------

struct PlaneCgArgs {
    int nplanes, nframes;
    const int* plane_frame;     // [planes]
    const int* frame_plane0;    // [frames]
    const int* frame_planes;    // [frames]
    int m, lo;                  // Omega
    int kb, klo, tw;            // band [klo, klo + kb)^2, its column tile width
    float rs, alpha;
    const float2* tw2;          // [N1][N2]
    const float* P;             // [frames][n][n], column-tiled
    long long p_stride;
    const float* winv;          // [kb][kb] band of 1/w, column-tiled
    const float2* rho;          // [frames][m][m] linearisation point
    const float2* c;            // [planes][m][m] its coil maps
    float2* r_c;                // [planes][kb][kb] CG vectors on the band (column-tiled)
    float2* p_c;
    float2* q_c;                // W^{-H} E(conj(rho) v) on the band
    float2* x_c;                // the solution's chat part (takes a p directly)
    float2* r_r;                // [frames][m][m]
    float2* p_r;
    float2* dx_r;
    float2* aux;                // [planes][m][m]
    double* part_g;             // k_plane_cg: [planes] |DF p|^2, then per plane |p_c|^2 and its
                                //   share of the frame's |p_r|^2 ([planes][2])
    double* part_r;             // update: [planes] |r_c|^2, [frames][rseg] |r_r|^2
    int rseg;                   // update: segments of a frame's rho part (kThreads elements)
    int first_iter;             // p = r
    ScalarStep fold;            // k_plane_cg: SC_RR0 / SC_RR; update: SC_GAMMA
    Scalars sc;
};

// the direction p = r + beta p, the same rounding in both kernels
__device__ __forceinline__ float2 cg_dir(float beta, float2 p, float2 r) {
    return make_float2(__fmaf_rn(beta, p.x, r.x), __fmaf_rn(beta, p.y, r.y));
}

template <int N>
__global__ __launch_bounds__(plane_threads(N)) void k_plane_cg(PlaneCgArgs a) {
    constexpr int NT = plane_threads(N);
    using Col = PlaneLines<N, 0>;
    using Row = PlaneLines<N, 1>;
    static_assert(plane_kernel_size(N), "whole-plane size");
    __shared__ float2 A[N * N];
    __shared__ float2 B[Col::BSIZE];
    __shared__ float2 TW[N];
    __shared__ double red[NT / 64];
    __shared__ float beta_sh;
    const int plane = blockIdx.x;
    if (plane >= a.nplanes) return;
    const int f = a.plane_frame[plane];
    const bool designated = plane == a.frame_plane0[f];
    const int m = a.m, lo = a.lo, kb = a.kb, klo = a.klo, tw = a.tw;
    const float rs = a.rs;
    const long long kbase = (long long)plane * kb * kb, cb = (long long)plane * m * m, fb = (long long)f * m * m;
    // the band's operands in flight before the scalar fold
    constexpr int MAXE = (N * N + NT - 1) / NT;
    float2 rv[MAXE], pv0[MAXE];
    float wv[MAXE];
    static_for<0, MAXE>([&](auto I) {
        const int e = (int)threadIdx.x + I * NT;
        if (e < kb * kb) {
            rv[I] = a.r_c[kbase + e];
            pv0[I] = a.first_iter ? rv[I] : a.p_c[kbase + e];
            wv[I] = a.winv[e];
        }
    });
    // beta of this iteration from the previous <r, r> (the frame's first plane records the step)
    if (threadIdx.x < 64) {
        const FrameScalars fs = load_frame_scalars(a.fold, a.sc, f);
        const double t = frame_total_wave(a.fold.g, a.fold.partial, f, a.frame_plane0, a.frame_planes);
        if (threadIdx.x == 0) {
            beta_sh = a.first_iter ? 0.f : cg_beta(a.fold, fs, t);
            if (designated) scalar_apply(a.fold, a.sc, f, t, fs);
        }
    }
    for (int e = threadIdx.x; e < N; e += NT) TW[e] = a.tw2[e];
    for (int e = threadIdx.x; e < N * N; e += NT) A[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float beta = beta_sh;
    // p = r + beta p on the band; W^{-1} p into the plane
    double acc = 0.0;
    static_for<0, MAXE>([&](auto I) {
        const int e = (int)threadIdx.x + I * NT;
        if (e < kb * kb) {
            const float2 pv = a.first_iter ? rv[I] : cg_dir(beta, pv0[I], rv[I]);
            a.p_c[kbase + e] = pv;
            acc += (double)(pv.x * pv.x + pv.y * pv.y);
            const int col = (e / (kb * tw)) * tw + e % tw, row = (e / tw) % kb;
            A[(klo + row) * N + klo + col] = cscale(pv, wv[I]);
        }
    });
    auto pr_of = [&](int q) -> float2 {   // the direction's rho part
        const float2 r = a.r_r[fb + q];
        return a.first_iter ? r : cg_dir(beta, a.p_r[fb + q], r);
    };
    // this plane's share of the frame's |p_r|^2 (p_r itself is written by the update)
    double ar = 0.0;
    {
        const int np = a.frame_planes[f], jj = plane - a.frame_plane0[f];
        const int chunk = (m * m + np - 1) / np, q1 = min(m * m, (jj + 1) * chunk);
        for (int q = jj * chunk + (int)threadIdx.x; q < q1; q += NT) {
            const float2 pv = pr_of(q);
            ar += (double)(pv.x * pv.x + pv.y * pv.y);
        }
    }
    {
        const double t = wg_sum<NT>(acc, red);
        const double tr = wg_sum<NT>(ar, red);
        if (threadIdx.x == 0) {
            a.part_g[a.nplanes + 2 * plane] = t;
            a.part_g[a.nplanes + 2 * plane + 1] = tr;
        }
    }
    auto in_om = [&](int i, int k) { return (unsigned)(i - lo) < (unsigned)m && (unsigned)(k - lo) < (unsigned)m; };
    auto colA = [&](int col, int row) -> float2& { return A[row * N + col]; };
    auto rowA = [&](int row, int col) -> float2& { return A[row * N + col]; };
    Col::template first<true, NT>(B, TW, [&](int col, int row) { return colA(col, row); });
    __syncthreads();
    Col::template second<true, NT>(B, rs, [&](int col, int row, float2 v) { colA(col, row) = v; });
    __syncthreads();
    Row::template first<true, NT>(B, TW, [&](int row, int col) { return rowA(row, col); });
    __syncthreads();
    Row::template middle<true, NT>(B, rs, [&](int row, int col, float2 dc) {
        if (!in_om(row, col)) return make_float2(0.f, 0.f);
        const int q = (row - lo) * m + (col - lo);
        return cadd(cmul(a.c[cb + q], pr_of(q)), cmul(a.rho[fb + q], dc));
    });
    __syncthreads();
    Row::template last<false, NT>(B, TW, rs, [&](int row, int col, float2 v) { rowA(row, col) = v; });
    __syncthreads();
    // columns: forward, P^2 with |P K|^2 = |DF p|^2 of the plane, inverse
    Col::template first<false, NT>(B, TW, [&](int col, int row) { return colA(col, row); });
    __syncthreads();
    const float* Pf = a.P + (long long)f * a.p_stride;
    double accg = 0.0;
    Col::template middle<false, NT>(B, rs, [&](int col, int row, float2 x) {
        const float p = Pf[((col / tw) * N + row) * tw + col % tw];
        accg += (double)(p * p * (x.x * x.x + x.y * x.y));
        return cscale(x, p * p);
    });
    __syncthreads();
    Col::template last<true, NT>(B, TW, rs, [&](int col, int row, float2 v) { colA(col, row) = v; });
    __syncthreads();
    Row::template first<true, NT>(B, TW, [&](int row, int col) { return rowA(row, col); });
    __syncthreads();
    Row::template middle<true, NT>(B, rs, [&](int row, int col, float2 v) {
        if (!in_om(row, col)) return make_float2(0.f, 0.f);
        const int q = (row - lo) * m + (col - lo);
        a.aux[cb + q] = cconjmul(a.c[cb + q], v);
        return cconjmul(a.rho[fb + q], v);
    });
    __syncthreads();
    Row::template last<false, NT>(B, TW, rs, [&](int row, int col, float2 v) { rowA(row, col) = v; });
    __syncthreads();
    // columns: forward; q = W^{-H} E(conj(rho) v) on the band
    Col::template first<false, NT>(B, TW, [&](int col, int row) { return colA(col, row); });
    __syncthreads();
    Col::template second<false, NT>(B, rs, [&](int col, int row, float2 v) {
        const int br = row - klo, bc = col - klo;
        if ((unsigned)br >= (unsigned)kb || (unsigned)bc >= (unsigned)kb) return;
        const int e = ((bc / tw) * kb + br) * tw + bc % tw;
        a.q_c[kbase + e] = cscale(v, a.winv[e]);
    });
    const double t = wg_sum<NT>(accg, red);
    if (threadIdx.x == 0) a.part_g[plane] = t;
}

// The update: blocks [0, planes) take a plane's band, blocks [planes,
// planes + frames * rseg) a segment of NT elements of a frame's rho part.
template <int NT>
__global__ __launch_bounds__(NT) void k_plane_cg_update(PlaneCgArgs a) {
    __shared__ double red[NT / 64];
    __shared__ float a_sh, beta_sh;
    const int b = blockIdx.x;
    const bool chat = b < a.nplanes;
    if (!chat && b >= a.nplanes + a.nframes * a.rseg) return;
    const int f = chat ? a.plane_frame[b] : (b - a.nplanes) / a.rseg;
    // a = rr / gamma (every block; the frame's first plane records it)
    if (threadIdx.x < 64) {
        const FrameScalars fs = load_frame_scalars(a.fold, a.sc, f);
        double t = frame_total_wave(a.fold.g, a.fold.partial, f, a.frame_plane0, a.frame_planes);
        const double t2 = frame_total_wave(a.fold.g2, a.fold.partial2, f, a.frame_plane0, a.frame_planes);
        if (threadIdx.x == 0) {
            t += (double)a.fold.alpha * t2;
            a_sh = cg_step(a.fold, fs, t);
            beta_sh = a.first_iter ? 0.f : a.sc.beta[f];
            if (chat && b == a.frame_plane0[f]) scalar_apply(a.fold, a.sc, f, t, fs);
        }
    }
    __syncthreads();
    const float av = a_sh, beta = beta_sh, al = a.alpha;
    double acc = 0.0;
    if (chat) {
        const long long kbase = (long long)b * a.kb * a.kb;
        for (int e = threadIdx.x; e < a.kb * a.kb; e += NT) {
            const float2 pv = a.p_c[kbase + e], qv = a.q_c[kbase + e];
            const float2 q = make_float2(qv.x + al * pv.x, qv.y + al * pv.y);   // N_alpha p
            float2 r = a.r_c[kbase + e];
            r.x -= av * q.x;
            r.y -= av * q.y;
            a.r_c[kbase + e] = r;
            float2 x = a.x_c[kbase + e];
            x.x += av * pv.x;
            x.y += av * pv.y;
            a.x_c[kbase + e] = x;
            acc += (double)(r.x * r.x + r.y * r.y);
        }
    } else {
        const int k = (b - a.nplanes) % a.rseg;
        const int E = a.m * a.m, e = k * NT + (int)threadIdx.x;
        if (e < E) {
            const long long fo = (long long)f * E;
            const float2 r0 = a.r_r[fo + e];
            const float2 pv = a.first_iter ? r0 : cg_dir(beta, a.p_r[fo + e], r0);
            // q = sum over the frame's coils of conj(c) v, plus alpha p (fixed order)
            const int p0 = a.frame_plane0[f], np = a.frame_planes[f];
            float2 s = make_float2(0.f, 0.f);
            for (int j = 0; j < np; ++j) s = cadd(s, a.aux[(long long)(p0 + j) * E + e]);
            const float2 q = make_float2(s.x + al * pv.x, s.y + al * pv.y);
            const float2 r = make_float2(r0.x - av * q.x, r0.y - av * q.y);
            float2 d = a.first_iter ? make_float2(0.f, 0.f) : a.dx_r[fo + e];
            d.x += av * pv.x;
            d.y += av * pv.y;
            a.p_r[fo + e] = pv;
            a.r_r[fo + e] = r;
            a.dx_r[fo + e] = d;
            acc = (double)(r.x * r.x + r.y * r.y);
        }
    }
    const double t = wg_sum<NT>(acc, red);
    if (threadIdx.x == 0) a.part_r[chat ? b : a.nplanes + (b - a.nplanes)] = t;
}

}  // namespace nlinv

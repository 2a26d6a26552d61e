// PCA channel compression (Sec. 3.2: before the reconstruction the receive
// channels are compressed by a principal component analysis, 32 to 8-12 in
// the paper's experiments):
//   covariance   A[i][k] = sum_m y_i[m] conj(y_k[m])          (J x J, Hermitian)
//   eigenpairs   A = V diag(lambda) V^H, lambda descending, each eigenvector's
//                largest-magnitude entry made real and positive (the first on a tie)
//   compression  y'_k[m] = sum_j conj(V[j][k]) y_j[m], k < K
// The covariance sums products of single-precision samples in FP64 (each
// product is exact there), per chunk of samples, then the chunks in a fixed
// order; the eigen-decomposition is a cyclic Jacobi method in FP64 inside one
// workgroup (disjoint pairs rotated together, round-robin order).
#pragma once
#include <hip/hip_runtime.h>

#include "cg_scalars.hpp"
#include "fft_core.hpp"

namespace nlinv {

constexpr int kPcaMaxJ = 64;
constexpr int kPcaChunk = 1024;        // samples per covariance partial (at least)
constexpr int kPcaMaxPartials = 1024;  // partials at most (larger chunks beyond)
constexpr int kPcaTile = 64;           // samples staged in LDS at a time
constexpr int kPcaMaxSweeps = 40;
constexpr int kPcaCompressK = 16;      // virtual channels per compression thread

struct PcaArgs {
    int J, K;
    long long M;
    int G;                         // covariance partials
    long long chunk;               // samples per partial (a multiple of kPcaTile)
    const float2* y;               // [J][M]
    double2* partial;              // [G][J][J]
    double2* A;                    // [J][J] covariance, then overwritten
    double* lambda;                // [J] eigenvalues, descending
    float2* V;                     // [J][K] kept eigenvectors (single precision)
    float2* y_out;                 // [K][M]
};

__device__ __forceinline__ double2 zmul_conj(float2 a, float2 b) {   // a conj(b) in FP64
    const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
    return make_double2(ax * bx + ay * by, ay * bx - ax * by);
}

// partial[g][i][k] = sum over chunk g of y_i conj(y_k), i <= k (the rest
// follows by symmetry); one workgroup per chunk
__global__ __launch_bounds__(kThreads) void k_pca_cov_partial(PcaArgs p) {
    __shared__ float2 tile[kPcaMaxJ * kPcaTile];
    const int J = p.J, g = blockIdx.x;
    const long long m0 = (long long)g * p.chunk, m1 = min(p.M, m0 + p.chunk);
    constexpr int kEnt = kPcaMaxJ * kPcaMaxJ / kThreads;   // entries per thread at most
    double2 acc[kEnt];
    for (int q = 0; q < kEnt; ++q) acc[q] = make_double2(0.0, 0.0);
    for (long long t0 = m0; t0 < m1; t0 += kPcaTile) {
        const int nt = (int)min((long long)kPcaTile, m1 - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < J * kPcaTile; e += kThreads) {
            const int j = e / kPcaTile, s = e % kPcaTile;
            tile[e] = s < nt ? p.y[(long long)j * p.M + t0 + s] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int q = 0; q < kEnt; ++q) {
            const int e = threadIdx.x + q * kThreads;
            if (e >= J * J) break;
            const int i = e / J, k = e % J;
            if (i > k) continue;
            const float2* yi = tile + i * kPcaTile;
            const float2* yk = tile + k * kPcaTile;
            double2 a = acc[q];
            for (int s = 0; s < nt; ++s) {
                const double2 z = zmul_conj(yi[s], yk[s]);
                a.x += z.x;
                a.y += z.y;
            }
            acc[q] = a;
        }
    }
    for (int q = 0; q < kEnt; ++q) {
        const int e = threadIdx.x + q * kThreads;
        if (e < J * J) p.partial[(long long)g * J * J + e] = acc[q];
    }
}

// A = the chunks' partials summed in chunk order; the lower triangle as the
// conjugate of the upper, the diagonal real: exactly Hermitian
__global__ __launch_bounds__(kThreads) void k_pca_cov_reduce(PcaArgs p) {
    const int J = p.J;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= J * J) return;
    const int i = e / J, k = e % J;
    const int eu = i <= k ? e : k * J + i;
    double2 s = make_double2(0.0, 0.0);
    for (int g = 0; g < p.G; ++g) {
        const double2 v = p.partial[(long long)g * J * J + eu];
        s.x += v.x;
        s.y += v.y;
    }
    if (i == k) s.y = 0.0;
    else if (i > k) s.y = -s.y;
    p.A[e] = s;
}

__device__ __forceinline__ double2 zmulf(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The eigen-decomposition of A (one workgroup).  Each step rotates the
// disjoint pairs of one round of a round-robin schedule: for the pair
// (p, q) with A[p][q] = |b| e^{i phi}, V = diag(1, e^{-i phi}) R, R the real
// rotation [[c, s], [-s, c]] with t = s/c the smaller root of
// t^2 - 2 tau t - 1 = 0, tau = (A[p][p] - A[q][q]) / (2 |b|), which zeroes
// A[p][q] in V^H A V.  A <- U^H A U and E <- E U with U the product of the
// step's rotations; sweeps until the off-diagonal part is below 1e-15 of A.
__global__ __launch_bounds__(kThreads) void k_pca_eig(PcaArgs p) {
    __shared__ double2 A[kPcaMaxJ * kPcaMaxJ];
    __shared__ double2 E[kPcaMaxJ * kPcaMaxJ];
    __shared__ double rc[kPcaMaxJ / 2], rs[kPcaMaxJ / 2];
    __shared__ double2 rph[kPcaMaxJ / 2];            // e^{-i phi} of each pair
    __shared__ int pp[kPcaMaxJ / 2], pq[kPcaMaxJ / 2];
    __shared__ double red[kThreads / 64];
    __shared__ int done;
    __shared__ int order[kPcaMaxJ];
    const int J = p.J, JJ = J * J;
    const int Jp = J + (J & 1);                       // a dummy index pads odd J
    for (int e = threadIdx.x; e < JJ; e += kThreads) {
        A[e] = p.A[e];
        E[e] = make_double2((e / J) == (e % J) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int sweep = 0; sweep < kPcaMaxSweeps; ++sweep) {
        // off-diagonal and total squared norms
        double off = 0.0, tot = 0.0;
        for (int e = threadIdx.x; e < JJ; e += kThreads) {
            const double v = A[e].x * A[e].x + A[e].y * A[e].y;
            tot += v;
            if ((e / J) != (e % J)) off += v;
        }
        const double toff = block_sum(off, red);
        const double ttot = block_sum(tot, red);
        if (threadIdx.x == 0) done = !(toff > 1e-30 * ttot);
        __syncthreads();
        if (done) break;
        for (int step = 0; step < Jp - 1; ++step) {
            // this step's pairs and their rotations
            if (threadIdx.x < Jp / 2) {
                const int i = threadIdx.x;
                auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + step) % (Jp - 1)); };
                int a = player(i), b = player(Jp - 1 - i);
                if (a > b) { const int t = a; a = b; b = t; }
                pp[i] = a;
                pq[i] = b;
                double c = 1.0, s = 0.0;
                double2 ph = make_double2(1.0, 0.0);
                if (b < J) {
                    const double2 apq = A[a * J + b];
                    const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                    if (mag > 0.0) {
                        const double tau = (A[a * J + a].x - A[b * J + b].x) / (2.0 * mag);
                        const double t = (tau >= 0.0 ? -1.0 : 1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        ph = make_double2(apq.x / mag, -apq.y / mag);   // e^{-i phi}
                    }
                }
                rc[i] = c;
                rs[i] = s;
                rph[i] = ph;
            }
            __syncthreads();
            // columns: A <- A U, E <- E U
            for (int e = threadIdx.x; e < (Jp / 2) * J; e += kThreads) {
                const int i = e / J, r = e % J;
                const int a = pp[i], b = pq[i];
                if (b >= J) continue;
                const double c = rc[i], s = rs[i];
                const double2 ph = rph[i];
                for (int w = 0; w < 2; ++w) {
                    double2* X = w == 0 ? A : E;
                    const double2 xa = X[r * J + a], xb = zmulf(X[r * J + b], ph);
                    X[r * J + a] = make_double2(c * xa.x - s * xb.x, c * xa.y - s * xb.y);
                    X[r * J + b] = make_double2(s * xa.x + c * xb.x, s * xa.y + c * xb.y);
                }
            }
            __syncthreads();
            // rows: A <- U^H A
            for (int e = threadIdx.x; e < (Jp / 2) * J; e += kThreads) {
                const int i = e / J, col = e % J;
                const int a = pp[i], b = pq[i];
                if (b >= J) continue;
                const double c = rc[i], s = rs[i];
                const double2 phc = make_double2(rph[i].x, -rph[i].y);   // e^{+i phi}
                const double2 xa = A[a * J + col], xb = zmulf(A[b * J + col], phc);
                A[a * J + col] = make_double2(c * xa.x - s * xb.x, c * xa.y - s * xb.y);
                A[b * J + col] = make_double2(s * xa.x + c * xb.x, s * xa.y + c * xb.y);
            }
            __syncthreads();
        }
    }
    // eigenvalues in descending order (ties keep the index order)
    if (threadIdx.x < J) {
        const int k = threadIdx.x;
        const double lk = A[k * J + k].x;
        int rank = 0;
        for (int i = 0; i < J; ++i) {
            const double li = A[i * J + i].x;
            rank += (li > lk) || (li == lk && i < k);
        }
        order[rank] = k;
    }
    __syncthreads();
    if (threadIdx.x < J) {
        const int r = threadIdx.x, k = order[r];
        p.lambda[r] = A[k * J + k].x;
        // phase: the largest-magnitude entry real and positive (first on a tie)
        int im = 0;
        double best = -1.0;
        for (int i = 0; i < J; ++i) {
            const double v = E[i * J + k].x * E[i * J + k].x + E[i * J + k].y * E[i * J + k].y;
            if (v > best) { best = v; im = i; }
        }
        const double mag = sqrt(best);
        const double2 fix = make_double2(E[im * J + k].x / mag, -E[im * J + k].y / mag);
        if (r < p.K)
            for (int i = 0; i < J; ++i) {
                const double2 v = zmulf(E[i * J + k], fix);
                p.V[i * p.K + r] = make_float2((float)v.x, (float)v.y);
            }
    }
}

// y'_k[m] = sum_j conj(V[j][k]) y_j[m]: one thread per sample and chunk of
// kPcaCompressK virtual channels
__global__ __launch_bounds__(kThreads) void k_pca_compress(PcaArgs p) {
    __shared__ float2 Vs[kPcaMaxJ * kPcaCompressK];
    const int k0 = blockIdx.y * kPcaCompressK, kn = min(kPcaCompressK, p.K - k0);
    for (int e = threadIdx.x; e < p.J * kPcaCompressK; e += kThreads) {
        const int j = e / kPcaCompressK, k = e % kPcaCompressK;
        Vs[e] = k < kn ? p.V[j * p.K + k0 + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const long long m = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (m >= p.M) return;
    float2 acc[kPcaCompressK];
    for (int k = 0; k < kPcaCompressK; ++k) acc[k] = make_float2(0.f, 0.f);
    for (int j = 0; j < p.J; ++j) {
        const float2 y = p.y[(long long)j * p.M + m];
        for (int k = 0; k < kPcaCompressK; ++k) {
            const float2 v = Vs[j * kPcaCompressK + k];
            acc[k].x += v.x * y.x + v.y * y.y;    // conj(v) y
            acc[k].y += v.x * y.y - v.y * y.x;
        }
    }
    for (int k = 0; k < kn; ++k) p.y_out[(long long)(k0 + k) * p.M + m] = acc[k];
}

}  // namespace nlinv

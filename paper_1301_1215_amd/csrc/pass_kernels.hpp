// Fused pass kernels of the NLINV operators (Schaetz & Uecker, Eqs. 2-3)
// for gfx950.
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
// row pass (axis 1), each a two-register-stage line FFT (fft_core.hpp) with
// the centring of Centre<N> and the unitary 1/sqrt(n) folded into its stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_scalars.hpp"
#include "coil_sum.hpp"
#include "fft_core.hpp"

namespace nlinv {

__device__ __forceinline__ float sgn(int i) { return (i & 1) ? -1.0f : 1.0f; }

// Centring.  With x' = x shifted by n/2, the centred DFT is the plain DFT of
// x' shifted by n/2 again: position p holds slot (p - n/2) mod n on both
// sides.  When N1 and N2 are even the shift is a compile-time permutation of
// the register index (k1 -> k1 + N1/2 on input, k2 -> k2 + N2/2 on output);
// otherwise the slot keeps its position and the checkerboard sign (-1)^p
// does the shift (the per-axis sign (-1)^(n/2) cancels on a square grid).
// SW: the transposed split N1 <-> N2 (a pass variant the autotuner can
// choose where N1 != N2); the twiddle table stays the one of the default
// split (its entry (a, b) is w_N^{ab}, symmetric in a and b).
// Whether the default split of an n-point line puts the stage-2 outputs of
// the centred half on compile-time slots (Centre<n>::HALF_BY_K2).
constexpr bool half_slots_k2(int n) {
    const int n1 = split_n1(n), n2 = n / n1;
    return n1 % 2 == 0 && n2 % 2 == 0 && n2 % 4 == 0 && (n / 4) % n1 == 0;
}

template <int N, bool SW = false>
struct Centre {
    static constexpr int N1 = SW ? N / split_n1(N) : split_n1(N), N2 = N / N1;
    static constexpr bool PERM = (N1 % 2 == 0) && (N2 % 2 == 0);
    // position of stage-1 input slot j2 + N2 k1
    static __device__ __forceinline__ int in_pos(int j2, int k1) {
        return PERM ? j2 + N2 * ((k1 + N1 / 2) % N1) : j2 + N2 * k1;
    }
    // position of stage-2 output slot k1 + N1 k2
    static __device__ __forceinline__ int out_pos(int k1, int k2) {
        return PERM ? k1 + N1 * ((k2 + N2 / 2) % N2) : k1 + N1 * k2;
    }
    static __device__ __forceinline__ float sign(int pos) { return PERM ? 1.0f : sgn(pos); }
    // With the permutation, N2 a multiple of 4 and N/4 a multiple of N1, the
    // stage-2 output slot k2 of every thread (any k1) lies in the centred half
    // [N/4, 3N/4) of the line exactly when k2' = (k2 + N2/2) mod N2 is in
    // [N2/4, 3 N2/4): which outputs fall in Omega = the centred half is then
    // known at compile time.
    static constexpr bool HALF_BY_K2 = PERM && N2 % 4 == 0 && (N / 4) % N1 == 0;
    static_assert(SW || HALF_BY_K2 == half_slots_k2(N), "host predicate");
    static constexpr bool half_k2(int k2) {
        const int k = (k2 + N2 / 2) % N2;
        return k >= N2 / 4 && k < 3 * N2 / 4;
    }
    // the i-th output slot in the centred half (N2/2 of them)
    static constexpr int half_k2_at(int i) {
        for (int k2 = 0; k2 < N2; ++k2)
            if (half_k2(k2) && i-- == 0) return k2;
        return -1;
    }
    // The same for the stage-1 input slots: with N1 a multiple of 4 and N/4
    // a multiple of N2, slot k1 (positions j2 + N2 k1', any j2) lies in the
    // centred half exactly when k1' = (k1 + N1/2) mod N1 is in [N1/4, 3 N1/4).
    static constexpr bool HALF_BY_K1 = PERM && N1 % 4 == 0 && (N / 4) % N2 == 0;
    static constexpr bool half_k1(int k1) {
        const int k = (k1 + N1 / 2) % N1;
        return k >= N1 / 4 && k < 3 * N1 / 4;
    }
};

// The band the solves keep of the sensitivities for the default weight
// (a = 220, l = 32): its side per grid size (the whole grid below 48).  The
// host derives the band from the weight itself; a CPU test checks that this
// table agrees, and a launch uses the compile-time geometry below only when
// its band is this one.
constexpr int default_band(int n) {
    switch (n) {
        case 48: case 64: case 96: return 32;
        case 128: case 192: return 64;
        case 256: return 96;
        case 384: return 128;
        case 512: return 160;
        case 768: return 224;
        case 1024: return 320;
        default: return n;
    }
}

// Compile-time geometry of the default band [KLO, KLO + KB) on a line of N
// (with the centring permutation and the bounds multiples of N1): stage-2
// output slot k2 of any thread lies in it exactly when k2' = (k2 + N2/2) mod
// N2 is in [KLO/N1, (KLO + KB)/N1); stage-1 input slot k1 (positions
// j2 + N2 k1') is wholly in it, wholly outside, or split by j2.
template <int N>
struct Band {
    using CT = Centre<N>;
    static constexpr int N1 = CT::N1, N2 = CT::N2;
    static constexpr int KB = default_band(N), KLO = (N - KB) / 2;
    static constexpr bool OK = CT::PERM && KB < N && KLO % N1 == 0 && KB % N1 == 0;
    static constexpr bool out_k2(int k2) {
        const int k = (k2 + N2 / 2) % N2;
        return k >= KLO / N1 && k < (KLO + KB) / N1;
    }
    static constexpr int NOUT = KB / N1;    // output slots per thread in the band
    static constexpr int out_k2_at(int i) {
        for (int k2 = 0; k2 < N2; ++k2)
            if (out_k2(k2) && i-- == 0) return k2;
        return -1;
    }
    // 0: every position of input slot k1 outside the band, 1: every one
    // inside, 2: split (decided per j2)
    static constexpr int in_k1(int k1) {
        const int r0 = N2 * ((k1 + N1 / 2) % N1), r1 = r0 + N2;
        if (r1 <= KLO || r0 >= KLO + KB) return 0;
        if (r0 >= KLO && r1 <= KLO + KB) return 1;
        return 2;
    }
};

// Inside a solve the n x n planes (CG vectors, data, P, 1/w) are stored
// column-tiled: [n / TW][n][TW], TW = 8 (4 when n is not a multiple of 8),
// so that a column pass reads and writes contiguous blocks instead of
// TW-wide row segments n apart.  A pass over L >= TW columns then covers
// whole tiles, hence whole cache lines: a tile wider than L would leave
// each line split between two workgroups, which fetch it twice.  The
// operator entry points take the plain row-major layout of the caller's
// arrays.
constexpr int plane_tile_width(int n) { return n % 8 == 0 ? 8 : 4; }
template <int N>
constexpr int plane_tile() { return plane_tile_width(N); }

template <int N>
__device__ __forceinline__ int big_idx(int r, int col, bool tiled) {
    constexpr int TW = plane_tile<N>();
    return tiled ? ((col / TW) * N + r) * TW + (col % TW) : r * N + col;
}

// Element i of an array that starts at a workgroup-uniform base and spans
// less than 4 GiB (one plane, one frame's rows): a 32-bit byte offset, which
// the compiler can address as scalar base + vector offset instead of
// forming a 64-bit address per access.
template <class T>
__device__ __forceinline__ T& elt(T* base, int i) {
    using B = std::conditional_t<std::is_const<T>::value, const char, char>;
    return *reinterpret_cast<T*>(reinterpret_cast<B*>(base) + (unsigned)i * (unsigned)sizeof(T));
}

// Load and store of an intermediate of the passes (T, T2; element i, as
// elt), read once by the pass that follows its producer.  With nt (the
// shape class's choice, made by the autotuner) both are non-temporal: the
// loads do not displace the operands that every iteration re-reads (coil
// maps, P, 1/w) from the L2, and the column passes' stores stream out
// instead of waiting dirty in one XCD's L2 for the write-back at the end of
// the kernel.  Where the intermediates are small enough to stay in the L2s
// between two passes, plain accesses are faster.
__device__ __forceinline__ float2 ld_mid(const float2* base, int i, bool nt) {
    using V = float __attribute__((ext_vector_type(2)));
    if (!nt) return elt(base, i);
    const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(&elt(base, i)));
    return make_float2(w.x, w.y);
}
__device__ __forceinline__ void st_mid(float2* base, int i, float2 v, bool nt) {
    using V = float __attribute__((ext_vector_type(2)));
    if (!nt) {
        elt(base, i) = v;
        return;
    }
    const V w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<V*>(&elt(base, i)));
}

// Outputs per chunk of a pointwise stage (a divisor of the stage length,
// at most cmax): the operands of a chunk are loaded together.
constexpr int pointwise_chunk(int n2, int cmax = 8) {
    for (int c = cmax; c > 1; --c)
        if (n2 % c == 0) return c;
    return 1;
}
// The row passes' products and the CG-update pass hold more operands per
// output; these chunk caps keep them at or under 128 VGPRs (4 waves per
// SIMD on gfx950), which measured faster than larger chunks at 3 waves.
constexpr int kRowChunk = 3;
constexpr int kCgChunk = 4;

// Threads of a pass workgroup over L lines: enough for one task per thread in
// the larger of the two FFT stages (L*N1 or L*N2 tasks), in whole wavefronts.
constexpr int pass_threads(int n, int L) {
    const int n1 = split_n1(n), n2 = n / n1;
    const int t = L * (n1 > n2 ? n1 : n2);
    return ((t + 63) / 64) * 64;
}

// ---------------------------------------------------------------------------
// column passes: a workgroup transforms L adjacent columns of one plane
// ---------------------------------------------------------------------------

enum ColMode : int {
    COL_WINV_IFFT_CROP = 0,   // T = crop_rows(IDFT_0(chat / w))
    COL_P_IFFT_CROP = 1,      // T = crop_rows(IDFT_0(P . z))
    COL_PAD_FFT_P = 2,        // out = P . DFT_0(pad_rows(T))
    COL_RESID_P_IFFT = 3,     // T = crop_rows(IDFT_0(P . (s_f y - P . DFT_0(pad_rows(T)))))  (in place):
                              //     the residual of F and the first step of its adjoint
    COL_PAD_FFT_P2_IFFT = 4,  // T = crop_rows(IDFT_0(P^2 . DFT_0(pad_rows(T))))   (in place)
    COL_PAD_FFT_WINV_ADD = 5, // out = DFT_0(pad_rows(T)) / w + a1_f add1 + a2_f add2
    COL_PAD_FFT_GPROD = 6,    // outR = Re(conj(g) . DFT_0(pad_rows(T)))  (mask gradient)
    COL_PUPD_WINV_IFFT_CROP = 7,   // CG: p = r + beta p (written back), then as COL_WINV_IFFT_CROP; |p|^2 partials
    COL_PAD_FFT_WINV_CG_UPD = 8,   // CG: q = DFT_0(pad_rows(T)) / w + alpha_f p (not stored);
                                   //     r -= a_f q, dx += a_f p; |r|^2 partials
};

struct ColArgs {
    const float2* in;
    float2* out;
    const float2* add1;       // RESID_P_IFFT: y; WINV_ADD: first added vector; GPROD: g
    const float2* add2;
    const float* P;           // [frames][n][n] with stride p_stride (0 = shared)
    long long p_stride;
    const int* plane_frame;   // nullable: all planes in frame 0
    const int* frame_plane0;  // nullable: one frame of nplanes planes
    const int* frame_planes;
    const float* s1;          // per-frame multiplier of add1 (nullable -> c1)
    const float* s2;
    float c1, c2;
    int m, lo;
    // The sensitivity-side modes (COL_WINV_IFFT_CROP, COL_PUPD_WINV_IFFT_CROP,
    // COL_PAD_FFT_WINV_ADD, COL_PAD_FFT_WINV_CG_UPD) act on the kb columns and
    // rows [kb_lo, kb_lo + kb) of k-space only: their chat-like operands and
    // 1/w are kb x kb arrays of that centred square, their T is [m][kb].
    // kb = n, kb_lo = 0 is the whole grid.
    int kb, kb_lo;
    int nplanes;
    int stream;               // intermediates T, T2 accessed non-temporally (ld_mid, st_mid)
    float rs;                 // 1/sqrt(n)
    const float2* tw2;        // [N1][N2]: exp(-2 pi i k1 j2 / n)
    const float* winv;        // [kb][kb]: 1/w, the inverse Sobolev weight on the band
    // COL_PUPD_WINV_IFFT_CROP: the direction update p = r + beta_f p is done
    // at load (in = p is rewritten); beta == nullptr means p = r.
    const float2* r_in;       // chat part of r (nullable: no update)
    float2* p_out;            // chat part of p
    const float* beta;
    float2* pr;               // rho part of p [frames][m*m], updated by the first plane of each frame
    const float2* rr;         // rho part of r
    // COL_PAD_FFT_WINV_CG_UPD: out = r (updated in place), add1 = p, s1 = alpha
    float2* dx;               // chat part of the accumulated step (x itself inside a solve)
    const float* cg_a;        // [frames] CG step a
    // FP64 partial sums, one per workgroup at partial[plane * tiles + tile]
    // (tiles = n / L), when non-null:
    //   COL_PUPD_WINV_IFFT_CROP   |p|^2 of the chat part at
    //                             partial[plane * 2 tiles + tile], and of this
    //                             workgroup's share of the frame's rho part at
    //                             partial[plane * 2 tiles + tiles + tile]
    //   COL_RESID_P_IFFT          |s y - P . DFT(...)|^2 (the residual's norm)
    //   COL_PAD_FFT_P2_IFFT       |P . DFT(...)|^2 = |DF h|^2 of the plane's coil
    //   COL_PAD_FFT_WINV_ADD      |out|^2
    //   COL_PAD_FFT_WINV_CG_UPD   |r|^2 after the update
    double* partial;
    int tiled;                // n x n planes, P and 1/w column-tiled (inside a solve)
    // COL_PAD_FFT_WINV_CG_UPD: the rho parts' CG update (a coil sum in its CG
    // form) runs as cs_blocks extra workgroups of the same launch, before the
    // column workgroups (the grid's first 8 * ceil(cs_blocks / 8) blocks, so
    // that they are dispatched first and the column tiles keep their XCD
    // assignment); it only needs the coil products and a, so it overlaps the
    // column work instead of taking a launch of its own
    CoilSumArgs cs;
    int cs_blocks;
    // COL_PUPD_WINV_IFFT_CROP: the previous iteration's SC_RR step folded in
    // (op SC_RR and partial set): every workgroup computes its frame's beta
    // from the <r, r> partials itself, and the frame's first workgroup
    // records it (beta is then not read from `beta`); or, before the first
    // iteration, the SC_RR0 step, recorded by the frame's first workgroup
    ScalarStep fold;
    Scalars sc;
    // COL_WINV_IFFT_CROP: rho_acc += rho_step on the rho parts [frames][m*m]
    // (the previous Newton step's rho update), done by the first plane's
    // workgroups of each frame, a chunk per column tile; nullable
    float2* rho_acc;
    const float2* rho_step;
};

// Work item w = tile * nplanes + plane (planes of a tile adjacent, so the P
// tile of a frame is reused); blocks are dealt to the 8 XCDs round robin, so
// block b runs item (b % 8) * per + b / 8: each XCD owns a contiguous range.
// `first` blocks of the grid (a multiple of 8) come before the work items.
__device__ __forceinline__ bool col_item(int ntiles, int nplanes, int& tile, int& plane, int first = 0) {
    const int total = ntiles * nplanes;
    const int per = (total + 7) / 8;
    const int b = (int)blockIdx.x - first;
    const int w = (b & 7) * per + (b >> 3);
    if (w >= total) return false;
    tile = w / nplanes;
    plane = w % nplanes;
    return true;
}

// TILED: the n x n operands are in the column-tiled solve layout (as
// ColArgs::tiled, fixed at compile time so no access computes both forms).
// HALF: Omega is the centred n/2 x n/2 block (a.m and a.lo are then ignored).
// BANDC: a sensitivity-side mode on the default band of Band<N> (a.kb and
// a.kb_lo are then ignored): which loads, stores and transform outputs fall
// in the band is known at compile time.
template <int N, int L, int MODE, bool TILED, bool HALF, bool BANDC = false>
__global__ __launch_bounds__(pass_threads(N, L)) void k_col(ColArgs a) {
    constexpr int NT = pass_threads(N, L);
    using CT = Centre<N>;
    constexpr int N1 = CT::N1, N2 = CT::N2;
    constexpr bool PSF = (MODE == COL_PAD_FFT_P2_IFFT);
    constexpr bool RESID = (MODE == COL_RESID_P_IFFT);
    constexpr bool TWO = PSF || RESID;             // forward, pointwise, inverse in one pass
    constexpr bool PUPD = (MODE == COL_PUPD_WINV_IFFT_CROP);
    constexpr bool WINV_IN = (MODE == COL_WINV_IFFT_CROP) || PUPD;
    constexpr bool INV1 = WINV_IN || (MODE == COL_P_IFFT_CROP);
    constexpr bool IN_CROP = !INV1;
    constexpr bool OUT_CROP = INV1 || TWO;
    constexpr bool CGU = (MODE == COL_PAD_FFT_WINV_CG_UPD);
    constexpr bool WINV_OUT = (MODE == COL_PAD_FFT_WINV_ADD) || CGU;
    constexpr bool RED = CGU || PUPD || TWO || (MODE == COL_PAD_FFT_WINV_ADD);  // can write partial sums
    // sensitivity-side modes work on the band of k-space (see ColArgs)
    constexpr bool CHAT = WINV_IN || WINV_OUT;
    constexpr int TW = plane_tile<N>();
    // Exchange buffer [k1][j2][l] (slot j2 + N2 k1 of line l), each k1 row
    // padded by L entries: the L-line groups of one wavefront then fall on
    // different LDS banks in every access pattern below.
    constexpr int RS = (N2 + 1) * L;               // k1 row stride
    __shared__ float2 bufA[N1 * RS];
    __shared__ double red[RED ? NT / 64 : 1];
    static_assert(NT % 64 == 0 && NT <= 1024, "pass workgroup size");

    using BD = Band<N>;
    static_assert(!BANDC || (CHAT && TILED && BD::OK), "compile-time band");
    const int kb = CHAT ? (BANDC ? BD::KB : a.kb) : N, klo = CHAT ? (BANDC ? BD::KLO : a.kb_lo) : 0;
    const int ncols = kb;                          // columns of this pass
    // element (grid row r, band column col) of a band-side array; whether
    // grid row r lies in the band
    auto cidx = [&](int r, int col) -> int {
        const int rc = r - klo;
        return TILED ? ((col / TW) * kb + rc) * TW + (col % TW) : rc * kb + col;
    };
    auto in_band = [&](int r) -> bool { return !CHAT || (unsigned)(r - klo) < (unsigned)kb; };
    // whether position r of stage-1 input slot K1 lies in the band (decided
    // at compile time with BANDC unless the slot is split by the band's edge)
    auto in_band_k1 = [&](auto K1, int r) -> bool {
        if constexpr (BANDC) {
            constexpr int st = BD::in_k1(decltype(K1)::value);
            if constexpr (st == 0) return false;
            else if constexpr (st == 1) return true;
            else return in_band(r);
        } else {
            return in_band(r);
        }
    };
    int first = 0;
    if constexpr (CGU) {
        first = 8 * ((a.cs_blocks + 7) / 8);
        if ((int)blockIdx.x < first) {
            if ((int)blockIdx.x < a.cs_blocks) coil_sum_block<NT>(a.cs, (int)blockIdx.x, red);
            return;
        }
    }
    int tile, plane;
    if (!col_item(ncols / L, a.nplanes, tile, plane, first)) return;
    const int col0 = tile * L;
    const int f = a.plane_frame ? a.plane_frame[plane] : 0;
    // HALF: Omega is the centred half of the grid (m = n/2, 2x oversampling),
    // fixed at compile time so that every crop and pad test folds away
    const int m = HALF ? N / 2 : a.m, lo = HALF ? N / 4 : a.lo;
    const float* P = a.P + (long long)f * a.p_stride;
    // plane offset of the input: T [m][ncols], a band array [kb][kb] or a grid plane
    const long long pofs = (long long)plane * (IN_CROP ? (long long)m * ncols : (long long)kb * kb);
    const float2* src = a.in + pofs;
    double acc = 0.0;     // this thread's share of the workgroup's partial sum
    double acc_rho = 0.0;
    bool first_plane = false;

    bool has_beta = false;
    float beta = 0.f;
    // PUPD: the first chunk of this thread's stage-1 operands, loaded before
    // beta is formed so that their latency overlaps the scalar fold
    constexpr int CHP = PUPD ? (BANDC ? N1 : pointwise_chunk(N1)) : 1;
    float2 rv0[CHP], pv0[CHP];
    float w0[CHP];
    int rho_e0 = 0, rho_e1 = 0;                    // PUPD: the rho-part chunk
    float2 rho_r0 = make_float2(0.f, 0.f), rho_p0 = rho_r0;   // and its first operands
    if constexpr (MODE == COL_WINV_IFFT_CROP) {
        if (a.rho_acc && (plane == 0 || (a.plane_frame && a.plane_frame[plane - 1] != f))) {
            const int E = m * m, ntiles = ncols / L;
            const int chunk = (E + ntiles - 1) / ntiles;
            const int e0 = tile * chunk, e1 = min(E, e0 + chunk);
            float2* x = a.rho_acc + (long long)f * E;
            const float2* d = a.rho_step + (long long)f * E;
            for (int e = e0 + threadIdx.x; e < e1; e += NT) x[e] = cadd(x[e], d[e]);
        }
    }
    if constexpr (PUPD) {
        // whether p = r + beta p or p = r is uniform and known from the
        // arguments; only beta's value waits for the fold
        const bool fold_rr = a.fold.partial && (a.fold.op == SC_RR || a.fold.op == SC_RR0);
        has_beta = fold_rr ? a.fold.op == SC_RR : a.beta != nullptr;
        static_assert(L * N2 <= NT, "one stage-1 task per thread");
        // this workgroup's chunk of the frame's rho part (see below) and the
        // operands of its first element per thread, also loaded before the fold
        {
            const int p0 = a.frame_plane0 ? a.frame_plane0[f] : 0;
            const int np = a.frame_planes ? a.frame_planes[f] : a.nplanes;
            const int E = m * m, ntiles = ncols / L, nch = np * ntiles;
            const int chunk = (E + nch - 1) / nch;
            rho_e0 = min(E, ((plane - p0) * ntiles + tile) * chunk);
            rho_e1 = min(E, rho_e0 + chunk);
            const int e = rho_e0 + (int)threadIdx.x;
            if (e < rho_e1) {
                rho_r0 = a.rr[(long long)f * E + e];
                rho_p0 = has_beta ? a.pr[(long long)f * E + e] : make_float2(0.f, 0.f);
            }
        }
        if ((int)threadIdx.x < L * N2) {
            const int l = threadIdx.x % L, j2 = threadIdx.x / L, col = col0 + l;
            static_for<0, CHP>([&](auto I) {
                constexpr int k1 = I;
                const int r = CT::in_pos(j2, k1);
                const float2 z = make_float2(0.f, 0.f);
                if (in_band_k1(std::integral_constant<int, k1>{}, r)) {
                    const int o = cidx(r, col);
                    rv0[I] = elt(a.r_in + pofs, o);
                    pv0[I] = has_beta ? elt(src, o) : z;
                    w0[I] = elt(a.winv, o);
                } else {
                    rv0[I] = z;
                    pv0[I] = z;
                    w0[I] = 0.f;
                }
            });
        }
        first_plane = plane == 0 || (a.plane_frame && a.plane_frame[plane - 1] != f);
        // uniform over the workgroup: SC_RR (iteration > 0) gives beta to
        // every workgroup; SC_RR0 (iteration 0, p = r) is only recorded, by
        // the frame's first workgroup
        const bool rr0 = a.fold.op == SC_RR0;
        const bool designated = first_plane && tile == 0;
        if (a.fold.partial && (a.fold.op == SC_RR || rr0)) {
            if (!rr0 || designated) {
                __shared__ float beta_sh;
                if (threadIdx.x < 64) {
                    const FrameScalars fs = load_frame_scalars(a.fold, a.sc, f);
                    const double t = frame_total_wave(a.fold.g, a.fold.partial, f, a.fold.frame_plane0,
                                                      a.fold.frame_planes);
                    if (threadIdx.x == 0) {
                        beta_sh = rr0 ? 0.f : cg_beta(a.fold, fs, t);
                        if (designated) scalar_apply(a.fold, a.sc, f, t, fs);
                    }
                }
                __syncthreads();
                if (!rr0) beta = beta_sh;
            }
        } else if (a.beta) {
            beta = a.beta[f];
        }
        // rho part of the direction update, shared by every workgroup of the
        // frame: chunk (coil, tile) of its J * tiles chunks
        {
            const int E = m * m;
            const float bf = beta;
            float2* pr = a.pr + (long long)f * E;
            const float2* rr = a.rr + (long long)f * E;
            for (int e = rho_e0 + threadIdx.x; e < rho_e1; e += NT) {
                const bool pre = e - rho_e0 < NT;   // operands loaded before the fold
                const float2 r = pre ? rho_r0 : rr[e];
                const float2 po = has_beta ? (pre ? rho_p0 : pr[e]) : make_float2(0.f, 0.f);
                const float2 pv = has_beta ? make_float2(r.x + bf * po.x, r.y + bf * po.y) : r;
                pr[e] = pv;
                acc_rho += (double)(pv.x * pv.x + pv.y * pv.y);
            }
        }
    }

    // ---- stage 1 of the first transform: positions in_pos(j2, k1) straight from HBM
    for (int t = threadIdx.x; t < L * N2; t += NT) {
        const int l = t % L, j2 = t / L, col = col0 + l;
        float2 v[N1];
        double pacc = 0.0;   // FP64 from the first term: these sums feed the CG scalars
        if constexpr (PUPD) {
            // p = r + beta p, written back; the operands of a chunk of
            // elements are loaded before its p values are stored (see the
            // last stage)
            constexpr int CH = CHP;
            auto chunks = [&](auto HASB) {
                constexpr bool HB = decltype(HASB)::value;
                const float b = HB ? beta : 0.f;
                static_for<0, N1 / CH>([&](auto C) {
                    float w[CH];
                    float2 rv[CH], pv[CH];
                    static_for<0, CH>([&](auto I) {
                        constexpr int k1 = C * CH + I;
                        if constexpr (decltype(C)::value == 0) {   // loaded before the fold
                            rv[I] = rv0[I];
                            pv[I] = pv0[I];
                            w[I] = w0[I];
                        } else {
                            const int r = CT::in_pos(j2, k1);
                            rv[I] = make_float2(0.f, 0.f);
                            pv[I] = rv[I];
                            w[I] = 0.f;
                            if (in_band_k1(std::integral_constant<int, k1>{}, r)) {
                                const int o = cidx(r, col);
                                rv[I] = elt(a.r_in + pofs, o);
                                if constexpr (HB) pv[I] = elt(src, o);
                                w[I] = elt(a.winv, o);
                            }
                        }
                    });
                    static_for<0, CH>([&](auto I) {
                        constexpr int k1 = C * CH + I;
                        const int r = CT::in_pos(j2, k1);
                        float2 x = rv[I];
                        if constexpr (HB) {
                            x.x += b * pv[I].x;
                            x.y += b * pv[I].y;
                        }
                        if (in_band_k1(std::integral_constant<int, k1>{}, r)) {
                            elt(a.p_out + pofs, cidx(r, col)) = x;
                            pacc += (double)(x.x * x.x + x.y * x.y);
                        }
                        v[k1] = cscale(x, CT::sign(r) * w[I]);
                    });
                });
            };
            if (has_beta) chunks(std::true_type{});
            else chunks(std::false_type{});
        } else {
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                const int r = CT::in_pos(j2, k1);
                float2 x = make_float2(0.f, 0.f);
                if constexpr (IN_CROP && HALF && CT::HALF_BY_K1) {
                    // Omega rows by slot, known at compile time
                    if constexpr (CT::half_k1(k1)) x = cscale(ld_mid(src, (r - lo) * ncols + col, a.stream), CT::sign(r));
                } else if constexpr (IN_CROP) {
                    const int ri = r - lo;
                    if (ri >= 0 && ri < m) x = cscale(ld_mid(src, ri * ncols + col, a.stream), CT::sign(r));
                } else if constexpr (WINV_IN) {
                    if (in_band_k1(std::integral_constant<int, k1>{}, r)) {
                        const int o = cidx(r, col);
                        x = cscale(elt(src, o), CT::sign(r) * elt(a.winv, o));
                    }
                } else {   // COL_P_IFFT_CROP
                    const int o = big_idx<N>(r, col, TILED);
                    x = cscale(elt(src, o), CT::sign(r) * elt(P, o));
                }
                v[k1] = x;
            });
        }
        if constexpr (PUPD) acc += pacc;
        RegDFT<N1, INV1>::run(v);
        static_for<0, N1>([&](auto K) {
            constexpr int k1 = K;
            float2 x = v[k1];
            if constexpr (k1 > 0) {
                const float2 w = elt(a.tw2, k1 * N2 + j2);
                x = INV1 ? cmulc(x, w) : cmul(x, w);
            }
            bufA[k1 * RS + j2 * L + l] = x;
        });
    }
    __syncthreads();

    if constexpr (TWO) {
        // The forward's stage 2, the pointwise step and the inverse's first
        // stage in one task: the inverse is the adjoint of the forward's
        // stages taken in reverse order (an N2-point inverse DFT over k2 in
        // the same registers), so the task writes its results back to the
        // very slots it read (no barrier in between); the last stage applies
        // the conjugate twiddle and the adjoint of stage 1 (tasks j2, outputs
        // at the stage-1 input positions).  The forward's raw outputs carry the
        // centring sign of their position on both sides of the pointwise
        // step, which the real pointwise factors leave unchanged.
        static_assert(L * N1 <= NT && L * N2 <= NT, "one task per thread");
        const float rs2 = a.rs * a.rs;
        {
            const int t = threadIdx.x;
            if (t < L * N1) {
                const int l = t % L, k1 = t / L, col = col0 + l;
                float2 v[N2];
                static_for<0, N2>([&](auto J) {
                    constexpr int j2 = J;
                    v[j2] = bufA[k1 * RS + j2 * L + l];
                });
                RegDFT<N2, false>::run(v);
                if constexpr (PSF) {   // times P^2 and 1/n
                    double kacc = 0.0;
                    static_for<0, N2>([&](auto K) {
                        constexpr int k2 = K;
                        const int r = CT::out_pos(k1, k2);
                        const float p = elt(P, big_idx<N>(r, col, TILED));
                        kacc += (double)(p * p * (v[k2].x * v[k2].x + v[k2].y * v[k2].y));
                        v[k2] = cscale(v[k2], p * p * rs2);
                    });
                    acc += kacc * (double)rs2;   // |P K|^2 with K = rs . v (unitary DFT)
                } else {               // residual q = s y - P K, then P q
                    const long long pb = (long long)plane * N * N;
                    const float sy = a.s1 ? a.s1[f] : a.c1;
                    constexpr int CH = pointwise_chunk(N2);
                    double racc = 0.0;
                    static_for<0, N2 / CH>([&](auto C) {
                        float w[CH];
                        float2 y[CH];
                        static_for<0, CH>([&](auto I) {
                            constexpr int k2 = C * CH + I;
                            const int o = big_idx<N>(CT::out_pos(k1, k2), col, TILED);
                            w[I] = elt(P, o);
                            y[I] = elt(a.add1 + pb, o);
                        });
                        static_for<0, CH>([&](auto I) {
                            constexpr int k2 = C * CH + I;
                            const float sg = CT::sign(CT::out_pos(k1, k2));
                            const float pk = w[I] * sg * a.rs;           // P times the forward's factors
                            const float2 q = make_float2(sy * y[I].x - pk * v[k2].x, sy * y[I].y - pk * v[k2].y);
                            racc += (double)(q.x * q.x + q.y * q.y);
                            v[k2] = cscale(q, w[I] * sg * a.rs);
                        });
                    });
                    acc += racc;
                }
                RegDFT<N2, true>::run(v);
                static_for<0, N2>([&](auto J) {
                    constexpr int j2 = J;
                    bufA[k1 * RS + j2 * L + l] = v[j2];
                });
            }
        }
        __syncthreads();
        // the conjugate twiddle, then the adjoint of stage 1: an N1-point
        // inverse DFT per j2, outputs at the positions the forward's stage-1
        // inputs came from
        const long long obase = (long long)plane * m * ncols;
        for (int t = threadIdx.x; t < L * N2; t += NT) {
            const int l = t % L, j2 = t / L, col = col0 + l;
            float2 v[N1];
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                v[k1] = bufA[k1 * RS + j2 * L + l];
                if constexpr (k1 > 0) v[k1] = cmulc(v[k1], elt(a.tw2, k1 * N2 + j2));
            });
            RegDFT<N1, true>::run(v);
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                const int r = CT::in_pos(j2, k1);
                if constexpr (HALF && CT::HALF_BY_K1) {
                    if constexpr (CT::half_k1(k1)) st_mid(a.out + obase, (r - lo) * ncols + col, cscale(v[k1], CT::sign(r)), a.stream);
                } else {
                    const int ri = r - lo;
                    if (ri >= 0 && ri < m) st_mid(a.out + obase, ri * ncols + col, cscale(v[k1], CT::sign(r)), a.stream);
                }
            });
        }
    }

    // ---- stage 2 of the last transform, straight to HBM (not in TWO modes,
    // which end above)
    constexpr bool INV2 = INV1;
    const long long pbase = (long long)plane * kb * kb;   // band or grid plane of the outputs
    const float s1 = a.s1 ? a.s1[f] : a.c1;
    const float s2 = a.s2 ? a.s2[f] : a.c2;
    const float av = CGU ? a.cg_a[f] : 0.f;
    if constexpr (!TWO) for (int t = threadIdx.x; t < L * N1; t += NT) {
        const int l = t % L, k1 = t / L, col = col0 + l;
        float2 v[N2];
        static_for<0, N2>([&](auto J) {
            constexpr int j2 = J;
            v[j2] = bufA[k1 * RS + j2 * L + l];
        });
        RegDFT<N2, INV2>::run(v);
        double facc = 0.0;
        if constexpr (OUT_CROP) {
            static_for<0, N2>([&](auto K) {
                constexpr int k2 = K;
                // HALF: the slots outside Omega are known at compile time
                if constexpr (!HALF || !CT::HALF_BY_K2 || CT::half_k2(k2)) {
                    const int rp = CT::out_pos(k1, k2);
                    const int ri = rp - lo;
                    if (ri >= 0 && ri < m) {
                        st_mid(a.out + (long long)plane * m * ncols, ri * ncols + col,
                               cscale(v[k2], CT::sign(rp) * a.rs), a.stream);
                    }
                }
            });
        } else {
            // The pointwise step over this thread's N2 outputs, CH at a time:
            // all operands of a chunk are loaded before any of its results is
            // stored.  (A store may alias a later operand as far as the
            // compiler can tell, so output-by-output code waits for each
            // output's loads in turn.)
            // BANDC: only the output slots in the band, all in one round
            constexpr int NOUT = BANDC ? BD::NOUT : N2;
            constexpr int CH = BANDC ? NOUT : pointwise_chunk(N2, CGU ? kCgChunk : 8);
            auto chunks = [&](auto HAS1, auto HAS2) {
                constexpr bool H1 = decltype(HAS1)::value, H2 = decltype(HAS2)::value;
                static_for<0, NOUT / CH>([&](auto C) {
                    float w[CH];
                    float2 u1[CH], u2[CH], u3[CH];
                    static_for<0, CH>([&](auto I) {
                        constexpr int k2 = BANDC ? BD::out_k2_at(C * CH + I) : C * CH + I;
                        const int rp = CT::out_pos(k1, k2);
                        if (BANDC || in_band(rp)) {
                            const int o = CHAT ? cidx(rp, col) : big_idx<N>(rp, col, TILED);
                            if constexpr (MODE == COL_PAD_FFT_P) w[I] = elt(P, o);
                            if constexpr (WINV_OUT || CGU) w[I] = elt(a.winv, o);
                            if constexpr (MODE == COL_PAD_FFT_GPROD || CGU || (WINV_OUT && H1))
                                u1[I] = elt(a.add1 + pbase, o);
                            if constexpr (WINV_OUT && H2) u2[I] = elt(a.add2 + pbase, o);
                            if constexpr (CGU) {
                                u2[I] = elt(a.out + pbase, o);    // r
                                u3[I] = elt(a.dx + pbase, o);
                            }
                        }
                    });
                    static_for<0, CH>([&](auto I) {
                        constexpr int k2 = BANDC ? BD::out_k2_at(C * CH + I) : C * CH + I;
                        const int rp = CT::out_pos(k1, k2);
                        if (!BANDC && !in_band(rp)) return;   // outside the band: not stored
                        const int o = CHAT ? cidx(rp, col) : big_idx<N>(rp, col, TILED);
                        float2 x = v[k2];
                        if constexpr (MODE == COL_PAD_FFT_P) {
                            elt(a.out + pbase, o) = cscale(x, CT::sign(rp) * a.rs * w[I]);
                        } else if constexpr (CGU) {
                            x = cscale(x, CT::sign(rp) * a.rs * w[I]);
                            const float2 u = u1[I];                          // p
                            x.x += s1 * u.x;                                 // q = N_alpha p
                            x.y += s1 * u.y;
                            float2 r = u2[I];
                            r.x -= av * x.x;
                            r.y -= av * x.y;
                            elt(a.out + pbase, o) = r;
                            float2 d = u3[I];
                            d.x += av * u.x;
                            d.y += av * u.y;
                            elt(a.dx + pbase, o) = d;
                            facc += (double)(r.x * r.x + r.y * r.y);
                        } else if constexpr (WINV_OUT) {
                            x = cscale(x, CT::sign(rp) * a.rs * w[I]);
                            if constexpr (H1) { x.x += s1 * u1[I].x; x.y += s1 * u1[I].y; }
                            if constexpr (H2) { x.x += s2 * u2[I].x; x.y += s2 * u2[I].y; }
                            elt(a.out + pbase, o) = x;
                            facc += (double)(x.x * x.x + x.y * x.y);
                        } else if constexpr (MODE == COL_PAD_FFT_GPROD) {
                            const float2 g = u1[I];
                            x = cscale(x, CT::sign(rp) * a.rs);
                            elt(reinterpret_cast<float*>(a.out) + pbase, o) = g.x * x.x + g.y * x.y;
                        }
                    });
                });
            };
            if constexpr (WINV_OUT) {
                if (a.add1 && a.add2) chunks(std::true_type{}, std::true_type{});
                else if (a.add1) chunks(std::true_type{}, std::false_type{});
                else if (a.add2) chunks(std::false_type{}, std::true_type{});
                else chunks(std::false_type{}, std::false_type{});
            } else {
                chunks(std::true_type{}, std::true_type{});
            }
        }
        acc += facc;
    }
    if constexpr (RED) {
        if (a.partial) {   // uniform over the workgroup
            const long long ntiles = ncols / L;
            const double t = wg_sum<NT>(acc, red);
            if constexpr (PUPD) {
                const double tr = wg_sum<NT>(acc_rho, red);
                if (threadIdx.x == 0) {
                    a.partial[(long long)plane * 2 * ntiles + tile] = t;
                    a.partial[(long long)plane * 2 * ntiles + ntiles + tile] = tr;
                }
            } else {
                if (threadIdx.x == 0) a.partial[(long long)plane * ntiles + tile] = t;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// row passes: a workgroup transforms L lines; line = (plane, Omega row i)
// ---------------------------------------------------------------------------

enum RowMode : int {
    ROW_CACHE = 0,   // c = crop_cols(IDFT_1(T))  (may fold a scalar step, see RowArgs); with out
                     // set also out = DFT_1(pad_cols(rho . c)) (as ROW_FWD), see RowArgs
    ROW_FWD = 1,     // T = DFT_1(pad_cols(rho . c))
    ROW_DERIV = 2,   // dc = crop_cols(IDFT_1(T)); T = DFT_1(pad_cols(drho . c + rho . dc))
    ROW_ADJ = 3,     // u = crop_cols(IDFT_1(T)); aux = conj(c) . u; T = DFT_1(pad_cols(conj(rho) . u))
};

struct RowArgs {
    const float2* in;        // T [planes][m][n], or [planes][m][kb] (ROW_CACHE, ROW_DERIV)
    float2* out;             // T [planes][m][n], or [planes][m][kb] (ROW_ADJ); may equal
                             // in when both have the same row length
    const float2* c;         // [planes][m][m]
    float2* c_out;           // ROW_CACHE output
    // ROW_CACHE with out set (Omega the centred half with compile-time slots,
    // half_slots_k2(n), the default split only): the pass continues as
    // ROW_FWD on the coil maps it has just formed, out = T of rho . c, so
    // that the forward model's first pass needs neither a launch of its own
    // nor a second read of c
    const float2* rho;       // [frames][m][m]
    const float2* drho;      // [frames][m][m]
    float2* aux;             // [planes][m][m]
    const int* plane_frame;
    int nlines;              // planes * m
    int m, lo;
    // band of k-space columns [kb_lo, kb_lo + kb) on the sensitivity side:
    // ROW_CACHE and ROW_DERIV read only those columns of their input (the
    // rest is zero), ROW_ADJ writes only those of its output
    int kb, kb_lo;
    int stream;              // the input T or T2 loaded non-temporally (ld_mid)
    float rs;
    const float2* tw2;       // [N1][N2]
    // ROW_ADJ with cgroup = 4 (Omega the centred half with compile-time
    // slots, L a multiple of 4, the four lines of a row's stage-2 tasks in one
    // wavefront, every frame's coil count a multiple of 4): a workgroup takes
    // L/4 rows of 4 consecutive coil planes, and aux receives the sum of the
    // four coils' products, [planes/4][m][m] (the coil sum then adds planes/4
    // partials per pixel)
    int cgroup;
    // ROW_ADJ, ROW_CACHE: a per-frame scalar step folded into the launch (op
    // SC_NONE or partial == nullptr: none), done by the first wavefront of
    // the first workgroups before their lines
    ScalarStep fold;
    Scalars sc;
};

template <int N, int L, int MODE, bool HALF, bool SW = false>
__global__ __launch_bounds__(pass_threads(N, L)) void k_row(RowArgs a) {
    using CT = Centre<N, SW>;
    constexpr int N1 = CT::N1, N2 = CT::N2;
    // twiddle w_N^{k1 j2} from the default split's table [N1d][N2d]
    auto twid = [&](int k1, int j2) -> float2 {
        if constexpr (SW) return elt(a.tw2, j2 * N1 + k1);
        else return elt(a.tw2, k1 * N2 + j2);
    };
    constexpr int NT = pass_threads(N, L);
    constexpr int S2 = N2 + 1;                      // padded stride of [line][k1][j2]
    static_assert(L * N1 <= NT && L * N2 <= NT, "one task per thread");
    // [line][k1][j2] (padded) for the stage exchange, or [line][pos] between
    // the two transforms: every stage reads into registers, waits, then writes
    __shared__ float2 buf[L * N1 * S2];
    // HALF: Omega is the centred half of the grid (m = n/2, 2x oversampling),
    // fixed at compile time so that every crop and pad test folds away
    const int m = HALF ? N / 2 : a.m, lo = HALF ? N / 4 : a.lo;
    // The workgroup's lines: L consecutive global lines (line = plane * m +
    // row), or with coil groups (RowArgs::cgroup) L/4 rows of 4 consecutive
    // coil planes, line ll the coil ll % 4 of row ll / 4; line ll sits at
    // global line line0 + loff(ll)
    constexpr bool CGROUP = MODE == ROW_ADJ && HALF && CT::HALF_BY_K2 && L % 4 == 0 && 64 % (4 * N1) == 0;
    const bool cg = CGROUP && a.cgroup == 4;
    int line0 = blockIdx.x * L, grp = 0;
    if (cg) {
        const int wpg = m / (L >= 4 ? L / 4 : 1);     // workgroups per coil group
        grp = blockIdx.x / wpg;
        line0 = grp * 4 * m + (blockIdx.x % wpg) * (L / 4);
    }
    auto loff = [&](int ll) { return cg ? (ll & 3) * m + (ll >> 2) : ll; };
    const int t = threadIdx.x;
    constexpr bool IN_BAND = MODE == ROW_CACHE || MODE == ROW_DERIV;   // input rows [kb]
    constexpr bool OUT_BAND = MODE == ROW_ADJ;                          // output rows [kb]
    const int kb = a.kb, klo = a.kb_lo;
    if constexpr (MODE == ROW_ADJ || MODE == ROW_CACHE) fold_scalar_step(a.fold, a.sc);

    if constexpr (MODE == ROW_FWD) {
        for (int idx = t; idx < L * N; idx += NT) {
            const int ll = idx / N, pos = idx % N;
            const int line = line0 + ll;
            const int q = pos - lo;
            float2 z = make_float2(0.f, 0.f);
            if (line < a.nlines && q >= 0 && q < m) {
                const int plane = line / m, i = line % m;
                const int f = a.plane_frame ? a.plane_frame[plane] : 0;
                z = cscale(cmul(elt(a.rho + (long long)f * m * m, i * m + q), elt(a.c + (long long)line0 * m, ll * m + q)),
                           CT::sign(pos));
            }
            buf[ll * N + pos] = z;
        }
        __syncthreads();
    } else {
        // inverse transform of the T rows: stage 1 from HBM
        if (t < L * N2) {
            const int ll = t / N2, j2 = t % N2;
            const int line = line0 + loff(ll);
            float2 v[N1];
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                const int p = CT::in_pos(j2, k1);
                v[k1] = make_float2(0.f, 0.f);
                if constexpr (IN_BAND) {
                    const int pc = p - klo;
                    if (line < a.nlines && (unsigned)pc < (unsigned)kb)
                        v[k1] = cscale(ld_mid(a.in + (long long)line0 * kb, loff(ll) * kb + pc, a.stream), CT::sign(p));
                } else {
                    if (line < a.nlines)
                        v[k1] = cscale(ld_mid(a.in + (long long)line0 * N, loff(ll) * N + p, a.stream), CT::sign(p));
                }
            });
            RegDFT<N1, true>::run(v);
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                float2 x = v[k1];
                if constexpr (k1 > 0) x = cmulc(x, twid(k1, j2));
                buf[(ll * N1 + k1) * S2 + j2] = x;
            });
        }
        __syncthreads();
        // stage 2, crop to Omega columns, pointwise products, zero-pad
        {
            const bool act = t < L * N1;
            const int ll = t / N1, k1 = t % N1;
            const int line = line0 + loff(ll);
            float2 v[N2];
            if (act) {
                static_for<0, N2>([&](auto J) {
                    constexpr int j2 = J;
                    v[j2] = buf[(ll * N1 + k1) * S2 + j2];
                });
                RegDFT<N2, true>::run(v);
                const bool live = line < a.nlines;
                // lines past the end read a valid line's operands (discarded)
                const int line_c = live ? line : a.nlines - 1;
                const int plane = line_c / m, i = line_c % m;
                const int f = a.plane_frame ? a.plane_frame[plane] : 0;
                if constexpr (MODE == ROW_CACHE) {
                    static_for<0, N2>([&](auto K) {
                        constexpr int k2 = K;
                        if constexpr (!HALF || !CT::HALF_BY_K2 || CT::half_k2(k2)) {
                            const int pos = CT::out_pos(k1, k2);
                            const int q = pos - lo;
                            if (live && q >= 0 && q < m)
                                elt(a.c_out + (long long)line0 * m, (line_c - line0) * m + q) =
                                    cscale(v[k2], CT::sign(pos) * a.rs);
                        }
                    });
                    if constexpr (HALF && CT::HALF_BY_K2) {
                        if (a.out) {   // fused forward: v = sign . rho . c on Omega, zero elsewhere
                            constexpr int NO = N2 / 2;
                            const float2* rrow = a.rho + ((long long)f * m + i) * m;
                            float2 rv[NO];
                            static_for<0, NO>([&](auto O) {
                                constexpr int k2 = CT::half_k2_at(O);
                                rv[O] = elt(rrow, CT::out_pos(k1, k2) - lo);
                            });
                            static_for<0, N2>([&](auto K) {
                                constexpr int k2 = K;
                                if constexpr (!CT::half_k2(k2)) v[k2] = make_float2(0.f, 0.f);
                            });
                            static_for<0, NO>([&](auto O) {
                                constexpr int k2 = CT::half_k2_at(O);
                                const int pos = CT::out_pos(k1, k2);
                                const float2 u = cscale(v[k2], CT::sign(pos) * a.rs);
                                v[k2] = live ? cscale(cmul(rv[O], u), CT::sign(pos)) : make_float2(0.f, 0.f);
                            });
                        }
                    }
                } else if constexpr (HALF && CT::HALF_BY_K2) {
                    // Omega = the centred half, its output slots known at
                    // compile time (N2/2 of them): their operands are loaded
                    // in one round (two for the derivative's three operands)
                    // before any product is formed or stored
                    constexpr int NO = N2 / 2;
                    constexpr int RCH = NO % 2 == 0 ? NO / 2 : NO;
                    const int cofs = (line_c - line0) * m;
                    const float2* crow = a.c + (long long)line0 * m;
                    const float2* rrow = a.rho + ((long long)f * m + i) * m;
                    const float2* drow = MODE == ROW_DERIV ? a.drho + ((long long)f * m + i) * m : nullptr;
                    static_for<0, N2>([&](auto K) {
                        constexpr int k2 = K;
                        if constexpr (!CT::half_k2(k2)) v[k2] = make_float2(0.f, 0.f);
                    });
                    // ROW_ADJ: the coil products of every round are stored
                    // after the last round's loads (a store between two load
                    // rounds would hold the second one back)
                    float2 aux[MODE == ROW_ADJ ? NO : 1];
                    static_for<0, NO / RCH>([&](auto R) {
                        float2 cv[RCH], rv[RCH], dv[RCH];
                        static_for<0, RCH>([&](auto I) {
                            constexpr int k2 = CT::half_k2_at(decltype(R)::value * RCH + I);
                            const int q = CT::out_pos(k1, k2) - lo;     // in [0, m)
                            cv[I] = elt(crow, cofs + q);
                            rv[I] = elt(rrow, q);
                            if constexpr (MODE == ROW_DERIV) dv[I] = elt(drow, q);
                        });
                        static_for<0, RCH>([&](auto I) {
                            constexpr int o = decltype(R)::value * RCH + I;
                            constexpr int k2 = CT::half_k2_at(o);
                            const int pos = CT::out_pos(k1, k2);
                            const float2 u = cscale(v[k2], CT::sign(pos) * a.rs);
                            float2 z;
                            if constexpr (MODE == ROW_DERIV) {
                                z = cadd(cmul(dv[I], cv[I]), cmul(rv[I], u));
                            } else {  // ROW_ADJ
                                aux[o] = cconjmul(cv[I], u);
                                z = cconjmul(rv[I], u);
                            }
                            v[k2] = live ? cscale(z, CT::sign(pos)) : make_float2(0.f, 0.f);
                        });
                    });
                    if constexpr (MODE == ROW_ADJ) {
                        if (CGROUP && cg) {
                            // the group's four coils sit N1 lanes apart in this
                            // wavefront: (c0 + c2) + (c1 + c3), stored by coil 0
                            float2* arow = a.aux + ((long long)grp * m + i) * m;
                            static_for<0, NO>([&](auto O) {
                                constexpr int k2 = CT::half_k2_at(O);
                                float2 x = aux[O];
                                x.x += __shfl_down(x.x, 2 * N1, 64);
                                x.y += __shfl_down(x.y, 2 * N1, 64);
                                x.x += __shfl_down(x.x, N1, 64);
                                x.y += __shfl_down(x.y, N1, 64);
                                if ((ll & 3) == 0 && live) elt(arow, CT::out_pos(k1, k2) - lo) = x;
                            });
                        } else if (live) {
                            static_for<0, NO>([&](auto O) {
                                constexpr int k2 = CT::half_k2_at(O);
                                elt(a.aux + (long long)line0 * m, cofs + (CT::out_pos(k1, k2) - lo)) = aux[O];
                            });
                        }
                    }
                } else {
                    // the pointwise products, CH outputs at a time: the operands
                    // of a chunk are loaded (from a valid column for outputs
                    // outside Omega) before any of its results is formed
                    constexpr int CH = pointwise_chunk(N2, kRowChunk);
                    // this line's row of c and aux from the workgroup's base, and its frame's row of rho
                    const int cofs = (line_c - line0) * m;
                    const float2* crow = a.c + (long long)line0 * m;
                    const float2* rrow = a.rho + ((long long)f * m + i) * m;
                    const float2* drow = MODE == ROW_DERIV ? a.drho + ((long long)f * m + i) * m : nullptr;
                    static_for<0, N2 / CH>([&](auto C) {
                        float2 cv[CH], rv[CH], dv[CH];
                        static_for<0, CH>([&](auto I) {
                            constexpr int k2 = C * CH + I;
                            const int q = CT::out_pos(k1, k2) - lo;
                            const int qc = (q >= 0 && q < m) ? q : 0;
                            cv[I] = elt(crow, cofs + qc);
                            rv[I] = elt(rrow, qc);
                            if constexpr (MODE == ROW_DERIV) dv[I] = elt(drow, qc);
                        });
                        static_for<0, CH>([&](auto I) {
                            constexpr int k2 = C * CH + I;
                            const int pos = CT::out_pos(k1, k2);
                            const int q = pos - lo;
                            float2 z = make_float2(0.f, 0.f);
                            if (live && q >= 0 && q < m) {
                                const float2 u = cscale(v[k2], CT::sign(pos) * a.rs);
                                if constexpr (MODE == ROW_DERIV) {
                                    z = cadd(cmul(dv[I], cv[I]), cmul(rv[I], u));
                                } else {  // ROW_ADJ
                                    elt(a.aux + (long long)line0 * m, cofs + q) = cconjmul(cv[I], u);
                                    z = cconjmul(rv[I], u);
                                }
                                z = cscale(z, CT::sign(pos));
                            }
                            v[k2] = z;
                        });
                    });
                }
            }
            if constexpr (MODE == ROW_CACHE) {
                if (!(HALF && CT::HALF_BY_K2) || !a.out) return;   // uniform over the workgroup
            }
            if constexpr (MODE == ROW_DERIV || MODE == ROW_ADJ || MODE == ROW_CACHE) {
                // The forward transform as the adjoint of the inverse's stages
                // in reverse order: the adjoint of stage 2 (an N2-point DFT)
                // on this task's registers, back into the slots it read
                // (v already carries the centring sign of its positions);
                // then the adjoint of stage 1 (twiddle, N1-point DFT) with
                // its outputs at the stage-1 input positions, straight to HBM
                if (act) {
                    RegDFT<N2, false>::run(v);
                    static_for<0, N2>([&](auto J) {
                        constexpr int j2 = J;
                        buf[(ll * N1 + k1) * S2 + j2] = v[j2];
                    });
                }
                __syncthreads();
                if (t < L * N2) {
                    const int lo2 = t / N2, j2 = t % N2;
                    if (line0 + loff(lo2) < a.nlines) {
                        float2 w[N1];
                        static_for<0, N1>([&](auto K) {
                            constexpr int kk = K;
                            w[kk] = buf[(lo2 * N1 + kk) * S2 + j2];
                            if constexpr (kk > 0) w[kk] = cmul(w[kk], twid(kk, j2));
                        });
                        RegDFT<N1, false>::run(w);
                        static_for<0, N1>([&](auto K) {
                            constexpr int kk = K;
                            const int pos = CT::in_pos(j2, kk);
                            const float2 x = cscale(w[kk], CT::sign(pos) * a.rs);
                            if constexpr (OUT_BAND) {
                                const int pc = pos - klo;
                                if ((unsigned)pc < (unsigned)kb)
                                    elt(a.out + (long long)line0 * kb, loff(lo2) * kb + pc) = x;
                            } else {
                                elt(a.out + (long long)line0 * N, loff(lo2) * N + pos) = x;
                            }
                        });
                    }
                }
                return;
            }
            __syncthreads();
            if (act) {
                static_for<0, N2>([&](auto K) {
                    constexpr int k2 = K;
                    if constexpr (!HALF || !CT::HALF_BY_K2 || CT::half_k2(k2)) {
                        const int pos = CT::out_pos(k1, k2);
                        // HALF: the positions outside Omega are never read below
                        if (!HALF || (pos >= lo && pos < lo + m)) buf[ll * N + pos] = v[k2];
                    }
                });
            }
        }
        __syncthreads();
    }
    // forward transform: stage 1 from the position-ordered lines
    {
        const bool act = t < L * N2;
        const int ll = t / N2, j2 = t % N2;
        float2 v[N1];
        if (act) {
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                const int pos = CT::in_pos(j2, k1);
                // HALF: the zero padding outside Omega is known at compile time
                v[k1] = (HALF && (pos < lo || pos >= lo + m)) ? make_float2(0.f, 0.f) : buf[ll * N + pos];
            });
            RegDFT<N1, false>::run(v);
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                if constexpr (k1 > 0) v[k1] = cmul(v[k1], twid(k1, j2));
            });
        }
        __syncthreads();
        if (act) {
            static_for<0, N1>([&](auto K) {
                constexpr int k1 = K;
                buf[(ll * N1 + k1) * S2 + j2] = v[k1];
            });
        }
    }
    __syncthreads();
    // stage 2 to HBM
    if (t < L * N1) {
        const int ll = t / N1, k1 = t % N1;
        const int line = line0 + ll;
        if (line < a.nlines) {
            float2 v[N2];
            static_for<0, N2>([&](auto J) {
                constexpr int j2 = J;
                v[j2] = buf[(ll * N1 + k1) * S2 + j2];
            });
            RegDFT<N2, false>::run(v);
            static_for<0, N2>([&](auto K) {
                constexpr int k2 = K;
                const int pos = CT::out_pos(k1, k2);
                if constexpr (OUT_BAND) {
                    const int pc = pos - klo;
                    if ((unsigned)pc < (unsigned)kb)
                        elt(a.out + (long long)line0 * kb, ll * kb + pc) = cscale(v[k2], CT::sign(pos) * a.rs);
                } else {
                    elt(a.out + (long long)line0 * N, ll * N + pos) = cscale(v[k2], CT::sign(pos) * a.rs);
                }
            });
        }
    }
}

}  // namespace nlinv

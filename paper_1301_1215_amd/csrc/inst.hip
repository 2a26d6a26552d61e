// Instantiation of the pass kernels for one grid size (NLINV_SIZE).
#include "launch.hpp"

#ifndef NLINV_SIZE
#error "build with -DNLINV_SIZE=<n>"
#endif

namespace nlinv {

// One column mode: the Omega-half and compile-time-band variants when the
// launch's geometry is theirs.
template <int N, int L, int MODE, bool T>
static void col_mode(const ColArgs& a, dim3 grid, dim3 block, hipStream_t s, bool half, bool bandc) {
    constexpr bool CHAT = MODE == COL_WINV_IFFT_CROP || MODE == COL_PUPD_WINV_IFFT_CROP ||
                          MODE == COL_PAD_FFT_WINV_ADD || MODE == COL_PAD_FFT_WINV_CG_UPD;
    if constexpr (T && CHAT && Band<N>::OK) {
        if (bandc) {
            if (half) hipLaunchKernelGGL((k_col<N, L, MODE, true, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_col<N, L, MODE, true, false, true>), grid, block, 0, s, a);
            return;
        }
    }
    if (T && half) hipLaunchKernelGGL((k_col<N, L, MODE, T, T>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_col<N, L, MODE, T, false>), grid, block, 0, s, a);
}

template <int N, int L>
static hipError_t col_L(int mode, const ColArgs& a, int nplanes, hipStream_t s) {
    // the sensitivity-side modes run over the kb columns of the band
    const bool chat = mode == COL_WINV_IFFT_CROP || mode == COL_PUPD_WINV_IFFT_CROP ||
                      mode == COL_PAD_FFT_WINV_ADD || mode == COL_PAD_FFT_WINV_CG_UPD;
    if (chat && (a.kb <= 0 || a.kb > N || a.kb % L != 0 || a.kb % plane_tile<N>() != 0 || a.kb_lo < 0 ||
                 a.kb_lo + a.kb > N))
        return hipErrorInvalidValue;
    const int ncols = chat ? a.kb : N;
    // 1D grid, a multiple of 8 blocks: the kernel deals work items to XCDs
    const int total = (ncols / L) * nplanes;
    // fused coil-sum workgroups, first in the grid (a multiple of 8 blocks)
    const int extra = mode == COL_PAD_FFT_WINV_CG_UPD ? 8 * ((a.cs_blocks + 7) / 8) : 0;
    const dim3 grid(8 * ((total + 7) / 8) + extra), block(pass_threads(N, L));
    const bool half = 2 * a.m == N && 4 * a.lo == N;
    const bool bandc = chat && a.kb == Band<N>::KB && a.kb_lo == Band<N>::KLO;
#define NLINV_COL(MODE, T) col_mode<N, L, MODE, T>(a, grid, block, s, half, bandc)
    if (a.tiled) {   // inside a solve: every mode, Omega = the centred half specialised
        switch (mode) {
            case COL_WINV_IFFT_CROP: NLINV_COL(COL_WINV_IFFT_CROP, true); break;
            case COL_P_IFFT_CROP: NLINV_COL(COL_P_IFFT_CROP, true); break;
            case COL_PAD_FFT_P: NLINV_COL(COL_PAD_FFT_P, true); break;
            case COL_RESID_P_IFFT: NLINV_COL(COL_RESID_P_IFFT, true); break;
            case COL_PAD_FFT_P2_IFFT: NLINV_COL(COL_PAD_FFT_P2_IFFT, true); break;
            case COL_PAD_FFT_WINV_ADD: NLINV_COL(COL_PAD_FFT_WINV_ADD, true); break;
            case COL_PAD_FFT_GPROD: NLINV_COL(COL_PAD_FFT_GPROD, true); break;
            case COL_PUPD_WINV_IFFT_CROP: NLINV_COL(COL_PUPD_WINV_IFFT_CROP, true); break;
            case COL_PAD_FFT_WINV_CG_UPD: NLINV_COL(COL_PAD_FFT_WINV_CG_UPD, true); break;
            default: return hipErrorInvalidValue;
        }
    } else {         // the operator entry points on row-major arrays
        switch (mode) {
            case COL_WINV_IFFT_CROP: NLINV_COL(COL_WINV_IFFT_CROP, false); break;
            case COL_P_IFFT_CROP: NLINV_COL(COL_P_IFFT_CROP, false); break;
            case COL_PAD_FFT_P: NLINV_COL(COL_PAD_FFT_P, false); break;
            case COL_PAD_FFT_P2_IFFT: NLINV_COL(COL_PAD_FFT_P2_IFFT, false); break;
            case COL_PAD_FFT_WINV_ADD: NLINV_COL(COL_PAD_FFT_WINV_ADD, false); break;
            case COL_PAD_FFT_GPROD: NLINV_COL(COL_PAD_FFT_GPROD, false); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef NLINV_COL
    return hipGetLastError();
}

template <int N, int L, bool SW>
static hipError_t row_L(int mode, const RowArgs& a, hipStream_t s) {
    if ((mode == ROW_CACHE || mode == ROW_DERIV || mode == ROW_ADJ) &&
        (a.kb <= 0 || a.kb > N || a.kb_lo < 0 || a.kb_lo + a.kb > N))
        return hipErrorInvalidValue;
    const dim3 grid((a.nlines + L - 1) / L), block(pass_threads(N, L));
    const bool half = 2 * a.m == N && 4 * a.lo == N;
    // the transposed split exists for the CG loop's row passes; the others
    // run the default split under every variant
#define NLINV_ROW_SPLIT(MODE, S)                                                          \
    if (half) hipLaunchKernelGGL((k_row<N, L, MODE, true, S>), grid, block, 0, s, a);      \
    else hipLaunchKernelGGL((k_row<N, L, MODE, false, S>), grid, block, 0, s, a)
#define NLINV_ROW(MODE) NLINV_ROW_SPLIT(MODE, SW)
    switch (mode) {
        case ROW_CACHE: NLINV_ROW_SPLIT(ROW_CACHE, false); break;
        case ROW_FWD: NLINV_ROW_SPLIT(ROW_FWD, false); break;
        case ROW_DERIV: NLINV_ROW(ROW_DERIV); break;
        case ROW_ADJ: NLINV_ROW(ROW_ADJ); break;
        default: return hipErrorInvalidValue;
    }
#undef NLINV_ROW
#undef NLINV_ROW_SPLIT
    return hipGetLastError();
}

template <int N>
hipError_t launch_col(int mode, int variant, const ColArgs& a, int nplanes, hipStream_t s) {
    if (nplanes <= 0) return hipSuccess;
    if constexpr (col_variant_ok(N, 0)) { if (variant == 0) return col_L<N, kColL[0]>(mode, a, nplanes, s); }
    if constexpr (col_variant_ok(N, 1)) { if (variant == 1) return col_L<N, kColL[1]>(mode, a, nplanes, s); }
    if constexpr (col_variant_ok(N, 2)) { if (variant == 2) return col_L<N, kColL[2]>(mode, a, nplanes, s); }
    if constexpr (col_variant_ok(N, 3)) { if (variant == 3) return col_L<N, kColL[3]>(mode, a, nplanes, s); }
    return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_row(int mode, int variant, const RowArgs& a, hipStream_t s) {
    if (a.nlines <= 0) return hipSuccess;
#define NLINV_RV(V)                                                                          \
    if constexpr (row_variant_ok(N, V)) {                                                    \
        if (variant == V) return row_L<N, row_lines(V), row_swapped(V)>(mode, a, s);         \
    }
    NLINV_RV(0) NLINV_RV(1) NLINV_RV(2) NLINV_RV(3) NLINV_RV(4) NLINV_RV(5) NLINV_RV(6) NLINV_RV(7)
#undef NLINV_RV
    return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_plane_normal(const PlaneArgs& a, hipStream_t s) {
    if constexpr (plane_kernel_size(N)) {
        if (a.nplanes <= 0) return hipSuccess;
        if (2 * a.lo + a.m != N || a.m <= 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_plane_normal<N>), dim3(a.nplanes), dim3(plane_threads(N)), 0, s, a);
        return hipGetLastError();
    } else {
        (void)a;
        (void)s;
        return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t launch_plane_cg(const PlaneCgArgs& a, hipStream_t s) {
    if constexpr (plane_kernel_size(N)) {
        if (a.nplanes <= 0) return hipSuccess;
        if (2 * a.lo + a.m != N || a.m <= 0 || a.kb <= 0 || a.klo < 0 || a.klo + a.kb > N || a.tw <= 0 ||
            a.kb % a.tw != 0 || a.rseg * kThreads < a.m * a.m)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_plane_cg<N>), dim3(a.nplanes), dim3(plane_threads(N)), 0, s, a);
        return hipGetLastError();
    } else {
        (void)a;
        (void)s;
        return hipErrorInvalidValue;
    }
}

template hipError_t launch_col<NLINV_SIZE>(int, int, const ColArgs&, int, hipStream_t);
template hipError_t launch_row<NLINV_SIZE>(int, int, const RowArgs&, hipStream_t);
template hipError_t launch_plane_normal<NLINV_SIZE>(const PlaneArgs&, hipStream_t);
template hipError_t launch_plane_cg<NLINV_SIZE>(const PlaneCgArgs&, hipStream_t);

}  // namespace nlinv

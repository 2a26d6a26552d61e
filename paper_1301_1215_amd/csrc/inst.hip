// Instantiation of the pass kernels for one grid size (NLINV_SIZE).
#include "launch.hpp"

#ifndef NLINV_SIZE
#error "build with -DNLINV_SIZE=<n>"
#endif

namespace nlinv {

template <int N, int L>
static hipError_t col_L(int mode, const ColArgs& a, int nplanes, hipStream_t s) {
    // 1D grid, a multiple of 8 blocks: the kernel deals work items to XCDs
    const int total = (N / L) * nplanes;
    const dim3 grid(8 * ((total + 7) / 8)), block(pass_threads(N, L));
    switch (mode) {
        case COL_WINV_IFFT_CROP: hipLaunchKernelGGL((k_col<N, L, COL_WINV_IFFT_CROP>), grid, block, 0, s, a); break;
        case COL_P_IFFT_CROP: hipLaunchKernelGGL((k_col<N, L, COL_P_IFFT_CROP>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_P: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_P>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_P_RESID: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_P_RESID>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_P2_IFFT: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_P2_IFFT>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_WINV_ADD: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_WINV_ADD>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_GPROD: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_GPROD>), grid, block, 0, s, a); break;
        case COL_PUPD_WINV_IFFT_CROP: hipLaunchKernelGGL((k_col<N, L, COL_PUPD_WINV_IFFT_CROP>), grid, block, 0, s, a); break;
        case COL_PAD_FFT_WINV_CG_UPD: hipLaunchKernelGGL((k_col<N, L, COL_PAD_FFT_WINV_CG_UPD>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int N, int L>
static hipError_t row_L(int mode, const RowArgs& a, hipStream_t s) {
    const dim3 grid((a.nlines + L - 1) / L), block(pass_threads(N, L));
    switch (mode) {
        case ROW_CACHE: hipLaunchKernelGGL((k_row<N, L, ROW_CACHE>), grid, block, 0, s, a); break;
        case ROW_FWD: hipLaunchKernelGGL((k_row<N, L, ROW_FWD>), grid, block, 0, s, a); break;
        case ROW_DERIV: hipLaunchKernelGGL((k_row<N, L, ROW_DERIV>), grid, block, 0, s, a); break;
        case ROW_ADJ: hipLaunchKernelGGL((k_row<N, L, ROW_ADJ>), grid, block, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
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
    if constexpr (row_variant_ok(N, 0)) { if (variant == 0) return row_L<N, kRowL[0]>(mode, a, s); }
    if constexpr (row_variant_ok(N, 1)) { if (variant == 1) return row_L<N, kRowL[1]>(mode, a, s); }
    if constexpr (row_variant_ok(N, 2)) { if (variant == 2) return row_L<N, kRowL[2]>(mode, a, s); }
    if constexpr (row_variant_ok(N, 3)) { if (variant == 3) return row_L<N, kRowL[3]>(mode, a, s); }
    return hipErrorInvalidValue;
}

template hipError_t launch_col<NLINV_SIZE>(int, int, const ColArgs&, int, hipStream_t);
template hipError_t launch_row<NLINV_SIZE>(int, int, const RowArgs&, hipStream_t);

}  // namespace nlinv

// Host-side launchers of the size-templated pass kernels.  Each grid size is
// instantiated in its own translation unit (inst.hip built with
// -DNLINV_SIZE=n) so that the sizes compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "pass_kernels.hpp"
#include "plane_kernel.hpp"

namespace nlinv {

// The grid sizes the library is built for: 2^p and 3 * 2^p from 8 to 1024.
#define NLINV_FOR_EACH_SIZE(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Pass variants: lines (columns or rows) per workgroup (its size follows
// from the lines and the line FFT split, pass_threads()).
constexpr int kColL[] = {16, 8, 32, 4};
constexpr int kRowL[] = {8, 16, 4, 2};
constexpr int kNumColVariants = 4;
constexpr int kNumRowVariants = 8;

constexpr bool col_variant_ok(int n, int v) {
    return v >= 0 && v < kNumColVariants && n % kColL[v] == 0 && n * kColL[v] <= 8192;
}
// Row variant v takes kRowL[v & 3] lines per workgroup; v >= 4 also
// transposes the line FFT's split N1 x N2 (only where N1 != N2) in the CG
// loop's row passes (the derivative and adjoint passes).
constexpr int row_lines(int v) { return kRowL[v & 3]; }
constexpr bool row_swapped(int v) { return v >= 4; }
constexpr bool row_variant_ok(int n, int v) {
    return v >= 0 && v < kNumRowVariants && n * row_lines(v) <= 8192 &&
           (!row_swapped(v) || split_n1(n) * split_n1(n) != n);
}

template <int N>
hipError_t launch_col(int mode, int variant, const ColArgs& a, int nplanes, hipStream_t s);
template <int N>
hipError_t launch_row(int mode, int variant, const RowArgs& a, hipStream_t s);
// the whole-plane normal operator and CG iteration (hipErrorInvalidValue
// where no such kernel exists)
template <int N>
hipError_t launch_plane_normal(const PlaneArgs& a, hipStream_t s);
template <int N>
hipError_t launch_plane_cg(const PlaneCgArgs& a, hipStream_t s);

#define NLINV_DECLARE(N)                                                                       \
    extern template hipError_t launch_col<N>(int, int, const ColArgs&, int, hipStream_t);       \
    extern template hipError_t launch_row<N>(int, int, const RowArgs&, hipStream_t);            \
    extern template hipError_t launch_plane_normal<N>(const PlaneArgs&, hipStream_t);            \
    extern template hipError_t launch_plane_cg<N>(const PlaneCgArgs&, hipStream_t);
NLINV_FOR_EACH_SIZE(NLINV_DECLARE)
#undef NLINV_DECLARE

}  // namespace nlinv

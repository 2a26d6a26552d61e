// Complex FFT building blocks for gfx950 (64-wide wavefronts, 256-thread
// workgroups): in-register DFTs of length R = 2^a 3^b <= 32 with
// compile-time twiddles, and the split N = N1 * N2 used by the pass kernels.
//
// A line of length N is transformed in two register stages around one LDS
// exchange ("four-step" decomposition of the DFT index):
//   X[k1 + N1 k2] = sum_{j2} w_N2^{j2 k2} . w_N^{j2 k1} . sum_{k1'} x[j2 + N2 k1'] w_N1^{k1' k1}
// stage 1: for each j2, an N1-point DFT of the elements j2 + N2 k1' held in
//          registers, times the twiddle w_N^{j2 k1} (a host-computed table);
// stage 2: for each k1, an N2-point DFT over j2 after the LDS exchange.
// The R-point register DFTs are decimation in time:
//   X[k + S q] = sum_{m<r} w_R^{m k} w_r^{m q} DFT_S(x[m + r i])[k],  R = r S.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace nlinv {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ---- compile-time twiddles ----------------------------------------------------

constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series, |x| <= pi: 30 terms are exact to double rounding
constexpr double ct_sin(double x) {
    double term = x, sum = x;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ct_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 30; ++k) {
        term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        sum += term;
    }
    return sum;
}
// angle 2 pi e / R reduced to (-pi, pi]
constexpr double ct_angle(int e, int R) {
    const int r = ((e % R) + R) % R;
    double a = 2.0 * kPi * (double)r / (double)R;
    return a > kPi ? a - 2.0 * kPi : a;
}

// a * exp(-+2 pi i E / R) (forward sign -, inverse +), trivial angles exact
template <int E, int R, bool INV>
__device__ __forceinline__ float2 twc(float2 a) {
    constexpr int e = ((E % R) + R) % R;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (2 * e == R) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * e == R) {
        return mul_mi<INV>(a);
    } else if constexpr (4 * e == 3 * R) {
        return mul_mi<!INV>(a);
    } else {
        constexpr float c = (float)ct_cos(ct_angle(e, R));
        constexpr float s = (float)(INV ? ct_sin(ct_angle(e, R)) : -ct_sin(ct_angle(e, R)));
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// ---- in-register DFTs (natural order in and out, unscaled) -------------------

template <int R, bool INV>
struct RegDFT;

template <bool INV>
struct RegDFT<1, INV> {
    static __device__ __forceinline__ void run(float2*) {}
};

template <bool INV>
struct RegDFT<2, INV> {
    static __device__ __forceinline__ void run(float2* v) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV>
struct RegDFT<3, INV> {
    static __device__ __forceinline__ void run(float2* v) {
        const float s3 = 0.86602540378443864676f;
        const float2 a = v[0], b = v[1], c = v[2];
        const float2 t = cadd(b, c), d = csub(b, c);
        const float2 m = make_float2(a.x - 0.5f * t.x, a.y - 0.5f * t.y);
        const float2 r = INV ? make_float2(-s3 * d.y, s3 * d.x) : make_float2(s3 * d.y, -s3 * d.x);
        v[0] = cadd(a, t);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    }
};

template <bool INV>
struct RegDFT<4, INV> {
    static __device__ __forceinline__ void run(float2* v) {
        const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const float2 s13 = cadd(v[1], v[3]), d13 = mul_mi<INV>(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    }
};

constexpr int reg_radix(int R) { return (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : 3; }

template <int R, bool INV>
struct RegDFT {
    static_assert(R <= 32 && R > 4, "register DFT length");
    static __device__ __forceinline__ void run(float2* v) {
        constexpr int r = reg_radix(R);
        constexpr int S = R / r;
        float2 sub[r][S];
        static_for<0, r>([&](auto M) {
            constexpr int m = M;
            static_for<0, S>([&](auto I) {
                constexpr int i = I;
                sub[m][i] = v[m + r * i];
            });
            RegDFT<S, INV>::run(sub[m]);
        });
        static_for<0, S>([&](auto K) {
            constexpr int k = K;
            float2 t[r];
            static_for<0, r>([&](auto M) {
                constexpr int m = M;
                t[m] = twc<m * k, R, INV>(sub[m][k]);
            });
            RegDFT<r, INV>::run(t);
            static_for<0, r>([&](auto Q) {
                constexpr int q = Q;
                v[k + S * q] = t[q];
            });
        });
    }
};

// ---- the split N = N1 * N2 ----------------------------------------------------

constexpr int split_n1(int n) {
    int best = 1;
    for (int d = 1; d * d <= n; ++d)
        if (n % d == 0 && d <= 32 && n / d <= 32) best = d;
    return best;
}

constexpr bool supported_len(int n) {
    if (n < 8 || n > 1024) return false;
    const int n1 = split_n1(n);
    if (n / n1 > 32) return false;
    int k = n;
    while (k % 2 == 0) k /= 2;
    while (k % 3 == 0) k /= 3;
    return k == 1;
}

}  // namespace nlinv

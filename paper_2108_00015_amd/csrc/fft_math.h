// Complex helpers and in-register radix-2/3/4/8/16 DFT butterflies shared by the
// FFT passes and the fused inverse-z / summation kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace conker {
namespace fftm {

template <typename T>
using cplx = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * (DIR i)
template <int DIR, typename C>
__device__ __forceinline__ C mul_di(C a) {
    if constexpr (DIR > 0) return C{-a.y, a.x};
    else return C{a.y, -a.x};
}

// X_k = sum_r v_r exp(DIR 2 pi i r k / R), in place.
template <int R, int DIR, typename C>
__device__ __forceinline__ void dft(C *v) {
    if constexpr (R == 2) {
        C a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (R == 3) {
        // w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2
        using T = decltype(v[0].x);
        const T s3 = (T)0.86602540378443864676 * (T)DIR;   // DIR sqrt(3)/2
        const C t = cadd(v[1], v[2]);
        const C d = csub(v[1], v[2]);
        const C m = C{v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y};
        v[0] = cadd(v[0], t);
        // X1 = m + i s3 d, X2 = m - i s3 d
        v[1] = C{m.x - s3 * d.y, m.y + s3 * d.x};
        v[2] = C{m.x + s3 * d.y, m.y - s3 * d.x};
    } else if constexpr (R == 4) {
        C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        C a2 = cadd(v[1], v[3]), a3 = mul_di<DIR>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    } else if constexpr (R == 16) {
        // even and odd halves as 8-point DFTs, odd ones turned by
        // exp(DIR 2 pi i k / 16), k = 0..7 (cos and sin of multiples of pi/8)
        using T = decltype(v[0].x);
        C e[8], o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        dft<8, DIR>(e);
        dft<8, DIR>(o);
        const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;   // cos, sin pi/8
        const T h = (T)0.70710678118654752440;
        const T d = (T)DIR;
        const T cs[8] = {(T)1, c1, h, s1, (T)0, -s1, -h, -c1};
        const T sn[8] = {(T)0, s1, h, c1, (T)1, c1, h, s1};
#pragma unroll
        for (int k = 1; k < 8; ++k) o[k] = cmul(o[k], C{cs[k], d * sn[k]});
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 8] = csub(e[k], o[k]);
        }
    } else {
        static_assert(R == 8, "radix");
        using T = decltype(v[0].x);
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        dft<4, DIR>(e);
        dft<4, DIR>(o);
        const T h = (T)0.70710678118654752440;   // 1/sqrt(2)
        const T d = (T)DIR;
        // o_k *= exp(DIR 2 pi i k / 8)
        o[1] = C{(o[1].x - d * o[1].y) * h, (o[1].y + d * o[1].x) * h};
        o[2] = mul_di<DIR>(o[2]);
        o[3] = C{(-o[3].x - d * o[3].y) * h, (d * o[3].x - o[3].y) * h};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

}  // namespace fftm
}  // namespace conker

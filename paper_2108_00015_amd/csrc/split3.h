// Three-term bfloat16 split of float32 operands for the matrix-core
// summations (contract.hip, fused.hip, fft.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace conker {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// One pair: the packed bfloat16 values of (a, b) (round to nearest even) and
// the floats they hold (low half shifted up, high half masked), so that one
// conversion serves both the operand and the residual.
__device__ __forceinline__ unsigned cvt2_bf16(float a, float b, float &fa, float &fb) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const unsigned u = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
    fa = __uint_as_float(u << 16);
    fb = __uint_as_float(u & 0xffff0000u);
    return u;
}

// x = h + m + l in bfloat16 terms: h = bf16(x), m = bf16(x - h), l = bf16(x - h - m).
__device__ __forceinline__ void split3(const float (&v)[8], bf16x8_t &hi, bf16x8_t &mi, bf16x8_t &lo) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    u32x4 h, m, l;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        float f0, f1, g0, g1, d0, d1;
        h[p] = cvt2_bf16(v[2 * p], v[2 * p + 1], f0, f1);
        const float r0 = v[2 * p] - f0, r1 = v[2 * p + 1] - f1;
        m[p] = cvt2_bf16(r0, r1, g0, g1);
        l[p] = cvt2_bf16(r0 - g0, r1 - g1, d0, d1);
    }
    hi = __builtin_bit_cast(bf16x8_t, h);
    mi = __builtin_bit_cast(bf16x8_t, m);
    lo = __builtin_bit_cast(bf16x8_t, l);
}

// acc += A^T B for a 16 x 16 tile over 32 cells in split-bfloat16 (the six
// products of order <= 2^-16: ll, mm, hl, mh, hm, hh, smallest first).
typedef float floatx4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void mma16_split3(floatx4_t &acc, const float (&a)[8], const float (&b)[8]) {
    bf16x8_t ah, am, al, bh, bm, bl;
    split3(a, ah, am, al);
    split3(b, bh, bm, bl);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
}

}  // namespace conker

// Split-precision parts shared by the MFMA kernels: x = hi + lo in bfloat16
// or half, products hi*hi + hi*lo + lo*hi accumulated in FP32 (the lo*lo
// term is dropped).
#pragma once

#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfi {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// 16x16x32 layout: A lane l holds A[l%16][8(l/16)+e], B lane l holds
// B[8(l/16)+e][l%16], e < 8; 16x16x16: 4(l/16)+e, e < 4 (checked by an
// in-bounds probe).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <int PREC> struct Split;

template <> struct Split<BF_BF16X3> {
    typedef bf16x8 v8;
    typedef shortx4 v4;
    typedef short e4;                        // element of v4
    static constexpr bool kScaled = false;   // bfloat16 has the FP32 range
    static __device__ __forceinline__ void put8(v8& h, v8& l, int e, float v) {
        const __bf16 hv = (__bf16)v;
        h[e] = hv;
        l[e] = (__bf16)(v - (float)hv);
    }
    static __device__ __forceinline__ void put4(v4& h, v4& l, int e, float v) {
        const __bf16 hv = (__bf16)v;
        const __bf16 lv = (__bf16)(v - (float)hv);
        h[e] = __builtin_bit_cast(short, hv);
        l[e] = __builtin_bit_cast(short, lv);
    }
    static __device__ __forceinline__ floatx4 mma32(v8 a, v8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ floatx4 mma16(v4 a, v4 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

template <> struct Split<BF_FP16X3> {
    typedef f16x8 v8;
    typedef f16x4 v4;
    typedef _Float16 e4;                     // element of v4
    static constexpr bool kScaled = true;    // half: scale each column
    static __device__ __forceinline__ void put8(v8& h, v8& l, int e, float v) {
        const _Float16 hv = (_Float16)v;
        h[e] = hv;
        l[e] = (_Float16)(v - (float)hv);
    }
    static __device__ __forceinline__ void put4(v4& h, v4& l, int e, float v) {
        const _Float16 hv = (_Float16)v;
        h[e] = hv;
        l[e] = (_Float16)(v - (float)hv);
    }
    static __device__ __forceinline__ floatx4 mma32(v8 a, v8 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ floatx4 mma16(v4 a, v4 b, floatx4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

}  // namespace bfi

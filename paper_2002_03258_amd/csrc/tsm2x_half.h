// The 16-bit storage formats of the precision form (bfloat16, binary16):
// round-to-nearest-even encoding of a float and the float value of an
// element, shared by the kernels that read or write the planes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsm {

enum { FMT_BF16 = 0, FMT_F16 = 1 };

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Round-to-nearest-even of a float to the 16-bit format, as its bit pattern.
template <int FMT>
__device__ __forceinline__ uint32_t rne16(float x) {
    if (FMT == FMT_BF16) {
        uint32_t u = __float_as_uint(x);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;   // NaN stays NaN
        u += 0x7fffu + ((u >> 16) & 1u);
        return u >> 16;
    } else {
        _Float16 h = (_Float16)x;                                       // v_cvt_f16_f32, RNE
        return (uint32_t)__builtin_bit_cast(uint16_t, h);
    }
}

template <int FMT>
__device__ __forceinline__ float val16(uint32_t h) {
    if (FMT == FMT_BF16) return __uint_as_float(h << 16);
    return (float)__builtin_bit_cast(_Float16, (uint16_t)h);
}

// Float value of the 16-bit element h (0: low half, 1: high half) of a dword.
template <int FMT>
__device__ __forceinline__ float half_val(uint32_t d, int h) {
    if (FMT == FMT_BF16) return __uint_as_float(h ? (d & 0xffff0000u) : (d << 16));
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(h ? (d >> 16) : (d & 0xffffu)));
}

}  // namespace tsm

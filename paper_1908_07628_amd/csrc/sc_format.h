// Split-complex ("SC") storage shared by the split GEMM and the kernels that write its operands:
// a row of Kpad complex values (Kpad % 4 == 0) is Kpad / 4 units of 32 bytes; unit u holds complex
// 4u .. 4u+3 as [hi: four u32 (re, im) half pairs][lo: four u32], x = hi + lo with hi = rn(x) and
// lo = rn(x - hi) in bf16 or fp16.  Offsets count 8-byte complex slots exactly as for complex64.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "eels.h"

namespace eels {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bf16 bits (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

template <int PREC>
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo) {
    if constexpr (PREC == EELS_BF16_SPLIT) {
        uint32_t ha = bf16_bits(a), hb = bf16_bits(b);
        float ra = a - __uint_as_float(ha << 16), rb = b - __uint_as_float(hb << 16);
        hi = ha | (hb << 16);
        lo = bf16_bits(ra) | (bf16_bits(rb) << 16);
    } else {
        _Float16 ha = (_Float16)a, hb = (_Float16)b;
        _Float16 la = (_Float16)(a - (float)ha), lb = (_Float16)(b - (float)hb);
        hi = (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
        lo = (uint32_t)__builtin_bit_cast(uint16_t, la) | ((uint32_t)__builtin_bit_cast(uint16_t, lb) << 16);
    }
}

__device__ __forceinline__ void sc_store(uint32_t* base, int64_t off, float2 v, int prec) {
    uint32_t hi, lo;
    if (prec == EELS_BF16_SPLIT) split2<EELS_BF16_SPLIT>(v.x, v.y, hi, lo);
    else split2<EELS_FP16_SPLIT>(v.x, v.y, hi, lo);
    int64_t u = off >> 2;
    int pos = (int)(off & 3);
    base[u * 8 + pos] = hi;
    base[u * 8 + 4 + pos] = lo;
}

}  // namespace eels

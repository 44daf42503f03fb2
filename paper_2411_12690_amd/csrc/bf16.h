// BF16 helpers for the reduced-precision reconstruction: round-to-nearest-even
// from FP32 (finite inputs), widening back to FP32, and the 16x16x32 MFMA
// operand type of CDNA4.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mos {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_widen(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// x ~= hi + lo with both halves BF16: the pair carries about 16 significant
// bits, so a product of two split operands kept to three terms
// (hi*hi + hi*lo + lo*hi) loses only ~2^-17 relative per term.
__device__ __forceinline__ void bf16_split(double x, uint16_t &hi, uint16_t &lo) {
    hi = bf16_rne((float)x);
    lo = bf16_rne((float)(x - (double)bf16_widen(hi)));
}

}  // namespace mos

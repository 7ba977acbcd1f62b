// pw_half.h -- 16-bit storage types.  Fields stored in 16 bits are widened to
// float for all arithmetic (the storage-reduction direction the paper's
// section 6 names for cutting memory traffic); results are rounded once to
// the storage type.
//   _Float16  IEEE binary16 (compiler type; conversions round to nearest even)
//   bf16_t    bfloat16: the upper 16 bits of an IEEE binary32, defined below
#pragma once
#include <hip/hip_runtime.h>

// Round-to-nearest-even of a binary32 to its upper 16 bits (bfloat16): add
// 0x7FFF plus the lowest kept bit, then truncate; NaNs stay NaN (quiet bit).
__host__ __device__ inline unsigned short bf16_bits_rne(float f)
{
    const unsigned x = __builtin_bit_cast(unsigned, f);
    if ((x & 0x7f800000u) == 0x7f800000u && (x & 0x007fffffu)) return (unsigned short)((x >> 16) | 0x0040u);
    return (unsigned short)((x + 0x7fffu + ((x >> 16) & 1u)) >> 16);
}

struct bf16_t {
    unsigned short bits;
    bf16_t() = default;
    __host__ __device__ constexpr explicit bf16_t(int zero_only) : bits((unsigned short)(zero_only * 0)) {}
    __host__ __device__ explicit bf16_t(float f) : bits(bf16_bits_rne(f)) {}
    // from double: rounded to float first, then to bfloat16 (the generator's
    // definition for 16-bit storage)
    __host__ __device__ explicit bf16_t(double d) : bits(bf16_bits_rne((float)d)) {}
    __host__ __device__ operator float() const { return __builtin_bit_cast(float, (unsigned)bits << 16); }
    __host__ __device__ explicit operator double() const { return (double)(float)*this; }
};

// Conversion of a generated double to a storage type.  Double goes to
// _Float16 through float as well, so that both 16-bit types share the
// generator's two-step definition; the float is pinned in a register so that
// the two conversions are not merged into one direct (singly rounded) one.
template <typename T>
__device__ inline T to_storage(double x) { return (T)x; }
template <>
__device__ inline _Float16 to_storage<_Float16>(double x)
{
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return (_Float16)f;
}
// Device rounding of a binary32 to bfloat16 with the compute unit's own
// conversion instruction: round to nearest even, the same bits as
// bf16_bits_rne for every value but NaN (any quiet NaN), in one instruction
// instead of the integer sequence.
__device__ __forceinline__ bf16_t bf16_from_float(float f)
{
    bf16_t y;
    y.bits = __builtin_bit_cast(unsigned short, (__bf16)f);
    return y;
}
template <>
__device__ inline bf16_t to_storage<bf16_t>(double x)
{
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return bf16_from_float(f);
}

// Rounding of an arithmetic-type result to the storage type, exactly once
// from the arithmetic type's value.  For binary16 the float result is pinned
// in a register first: otherwise the compiler may fold the last fused
// multiply-add and the conversion into one mixed-precision instruction that
// rounds the exact sum straight to 16 bits, which can differ in the last bit
// and would make the result depend on instruction selection.
template <typename T, typename C>
__device__ __forceinline__ T store_round(C x)
{
    return (T)x;
}
template <>
__device__ __forceinline__ _Float16 store_round<_Float16, float>(float x)
{
    asm volatile("" : "+v"(x));
    return (_Float16)x;
}
template <>
__device__ __forceinline__ bf16_t store_round<bf16_t, float>(float x)
{
    asm volatile("" : "+v"(x));
    return bf16_from_float(x);
}

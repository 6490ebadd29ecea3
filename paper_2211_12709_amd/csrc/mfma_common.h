// mfma_common.h -- fragment conventions shared by the MFMA kernels.
//
// All MFMA work uses 16x16 output tiles.  One "K chunk" is 16 deep: lane
// l = 16 g + c (g = l / 16, c = l % 16) holds 4 consecutive K values
// k = 16 q + 4 g + j (j = 0..3) of row c of the A tile and of column c of the
// B tile.  For bfloat16 operands that is exactly one v_mfma_f32_16x16x16_bf16;
// for float operands it is four v_mfma_f32_16x16x4_f32, the j-th one taking
// value j of each lane (its K row g is then k = 16 q + 4 g + j, a fixed
// permutation that A and B share, so the sum over k is unchanged).
// An accumulator tile holds C[4 g + r][c] in element r, so the 4 rows a lane
// owns in a 16-row output tile are exactly the 4 K values it needs when that
// tile becomes the next product's K chunk: chained products never move data
// between lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace fno {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

typedef short s2v __attribute__((ext_vector_type(2)));

// Element type of an intermediate complex spectrum handed to a kernel working in type T:
// (re, im) float for float, (re, im) bfloat16 bits for bfloat16.
template <typename T> struct CplxOf;
template <> struct CplxOf<float> { typedef float2 type; };
template <> struct CplxOf<__bf16> { typedef s2v type; };

// Operand fragment type of the MFMA for activation/compute type T.
template <typename T> struct OpOf;
template <> struct OpOf<float> { typedef f4v type; };
template <> struct OpOf<__bf16> { typedef s4v type; };

__device__ __forceinline__ f4v mma16(f4v a, f4v b, f4v acc)
{
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
    return acc;
}

__device__ __forceinline__ f4v mma16(s4v a, s4v b, f4v acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}

// Two K chunks in one product: acc + a0 b0 + a1 b1.  For bfloat16 one v_mfma_f32_16x16x32_bf16,
// whose 8 K values per lane are taken as the two chunks' 4 + 4 (a fixed permutation of K shared by
// A and B, so the sum over K is unchanged); for float the two chunk products.
typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v_ __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4v mma32(s4v a0, s4v a1, s4v b0, s4v b1, f4v acc)
{
    const s8v a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const s8v b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8v_, a), __builtin_bit_cast(b8v_, b), acc, 0, 0,
                                                   0);
}
__device__ __forceinline__ f4v mma32(f4v a0, f4v a1, f4v b0, f4v b1, f4v acc) { return mma16(a1, b1, mma16(a0, b0, acc)); }

__device__ __forceinline__ short bf16_bits(float v) { return __builtin_bit_cast(short, (__bf16)v); }

// Two floats -> two bfloat16 (round to nearest even) in one 32-bit word, a in the low half: one
// v_cvt_pk_bf16_f32 (converting the halves one at a time leaves a repack per pair).
typedef float f2v_ __attribute__((ext_vector_type(2)));
typedef __bf16 b2v_ __attribute__((ext_vector_type(2)));
typedef unsigned u2v_ __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned bf16_pack2(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f2v_{a, b}, b2v_));
}
__device__ __forceinline__ s4v bf16_pack4(float a, float b, float c, float d)
{
    return __builtin_bit_cast(s4v, u2v_{bf16_pack2(a, b), bf16_pack2(c, d)});
}

// Accumulator (4 floats) -> operand fragment of type T.
template <typename T> __device__ __forceinline__ typename OpOf<T>::type to_op(f4v v);
template <> __device__ __forceinline__ f4v to_op<float>(f4v v) { return v; }
template <> __device__ __forceinline__ s4v to_op<__bf16>(f4v v) { return bf16_pack4(v[0], v[1], v[2], v[3]); }

template <typename T> __device__ __forceinline__ typename OpOf<T>::type op_zero();
template <> __device__ __forceinline__ f4v op_zero<float>() { return f4v{0.f, 0.f, 0.f, 0.f}; }
template <> __device__ __forceinline__ s4v op_zero<__bf16>() { return s4v{0, 0, 0, 0}; }

__device__ __forceinline__ f4v f4_zero() { return f4v{0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ f4v op_zero_of(f4v) { return f4_zero(); }
__device__ __forceinline__ s4v op_zero_of(s4v) { return s4v{0, 0, 0, 0}; }

// Value of lane (l & ~15) | ((l + 8) & 15): rotate each row of 16 lanes by 8 (DPP row_ror:8).
__device__ __forceinline__ float row_ror8(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
}

// Element j of a fragment as float.
__device__ __forceinline__ float op_get(f4v v, int j) { return v[j]; }
__device__ __forceinline__ float op_get(s4v v, int j)
{
    return __uint_as_float(((unsigned)(unsigned short)v[j]) << 16);
}


template <typename T> __device__ __forceinline__ typename OpOf<T>::type op_neg(typename OpOf<T>::type v);
template <> __device__ __forceinline__ f4v op_neg<float>(f4v v) { return -v; }
template <> __device__ __forceinline__ s4v op_neg<__bf16>(s4v v)
{
    return s4v{(short)(v[0] ^ (short)0x8000), (short)(v[1] ^ (short)0x8000), (short)(v[2] ^ (short)0x8000),
               (short)(v[3] ^ (short)0x8000)};
}

template <typename T> __device__ __forceinline__ typename OpOf<T>::type op_from4(float a, float b, float c, float d);
template <> __device__ __forceinline__ f4v op_from4<float>(float a, float b, float c, float d) { return f4v{a, b, c, d}; }
template <> __device__ __forceinline__ s4v op_from4<__bf16>(float a, float b, float c, float d)
{
    return bf16_pack4(a, b, c, d);
}

// Store element j of a fragment to *p (its storage type, bits unchanged).
__device__ __forceinline__ void op_put(float *p, f4v v, int j) { *p = v[j]; }
__device__ __forceinline__ void op_put(__bf16 *p, s4v v, int j) { *reinterpret_cast<short *>(p) = v[j]; }

// 4 consecutive activations as floats (vector load).
__device__ __forceinline__ void load4(const float *p, float (&v)[4])
{
    const f4v t = *reinterpret_cast<const f4v *>(p);
    v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
}
__device__ __forceinline__ void load4(const __bf16 *p, float (&v)[4])
{
    const s4v t = *reinterpret_cast<const s4v *>(p);
    v[0] = op_get(t, 0); v[1] = op_get(t, 1); v[2] = op_get(t, 2); v[3] = op_get(t, 3);
}
__device__ __forceinline__ void store4(float *p, const float (&v)[4])
{
    *reinterpret_cast<f4v *>(p) = f4v{v[0], v[1], v[2], v[3]};
}
__device__ __forceinline__ void store4(__bf16 *p, const float (&v)[4])
{
    *reinterpret_cast<s4v *>(p) = bf16_pack4(v[0], v[1], v[2], v[3]);
}

// A fragment (or any vector) from / to global memory that is only 4-byte aligned: a multi-dword
// access at dword alignment, which the target's global memory model allows (rows of an even
// number of bfloat16 values start on 4 bytes, not on the vector's own size).
template <typename V, typename E> __device__ __forceinline__ V ld_dword_aligned(const E *p)
{
    V v;
    __builtin_memcpy(&v, p, sizeof(V));
    return v;
}
template <typename V, typename E> __device__ __forceinline__ void st_dword_aligned(E *p, const V &v)
{
    __builtin_memcpy(p, &v, sizeof(V));
}

// 4x4 transpose: r[j] = {v[0][j], v[1][j], v[2][j], v[3][j]} (element j of four fragments).
__device__ __forceinline__ void op_transpose4(const f4v (&v)[4], f4v (&r)[4])
{
#pragma unroll
    for (int j = 0; j < 4; j++) r[j] = f4v{v[0][j], v[1][j], v[2][j], v[3][j]};
}
__device__ __forceinline__ void op_transpose4(const s4v (&v)[4], s4v (&r)[4])
{
#pragma unroll
    for (int j = 0; j < 4; j++) r[j] = s4v{v[0][j], v[1][j], v[2][j], v[3][j]};
}

// 8 consecutive activations <-> two fragments (one 16-byte access for bfloat16, two for float).
__device__ __forceinline__ void load8(const float *p, f4v &a, f4v &b)
{
    a = *reinterpret_cast<const f4v *>(p);
    b = *reinterpret_cast<const f4v *>(p + 4);
}
__device__ __forceinline__ void load8(const __bf16 *p, s4v &a, s4v &b)
{
    const s8v t = *reinterpret_cast<const s8v *>(p);
    a = s4v{t[0], t[1], t[2], t[3]};
    b = s4v{t[4], t[5], t[6], t[7]};
}
__device__ __forceinline__ void store8(float *p, const float (&v)[2][4])
{
    *reinterpret_cast<f4v *>(p) = f4v{v[0][0], v[0][1], v[0][2], v[0][3]};
    *reinterpret_cast<f4v *>(p + 4) = f4v{v[1][0], v[1][1], v[1][2], v[1][3]};
}
__device__ __forceinline__ void store8(__bf16 *p, const float (&v)[2][4])
{
    typedef unsigned u4v_ __attribute__((ext_vector_type(4)));
    *reinterpret_cast<u4v_ *>(p) = u4v_{bf16_pack2(v[0][0], v[0][1]), bf16_pack2(v[0][2], v[0][3]),
                                        bf16_pack2(v[1][0], v[1][1]), bf16_pack2(v[1][2], v[1][3])};
}

}  // namespace fno

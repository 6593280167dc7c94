// DFT stages as matrix-core products for the four-byte (FP16 / BF16) storage path.
//
// A radix-R DFT applied to a batch of vectors is a complex matrix product, and a
// complex product is a real one on [re, im] pairs.  The stages here use gfx950's
// v_mfma_f32_32x32x16_{f16,bf16}: D (32x32, FP32) += A (32x16) B (16x32), each lane
// holding 8 consecutive K values of one row of A (lane l: row l%32, K 8(l/32)..+7),
// 8 of one column of B (column l%32, the same K range) and 16 values of D (column
// l%32, rows 8(v/4) + 4(l/32) + v%4 for v < 16).
//
// Complex operands are interleaved along K: real K index 2n + c is part c (0 re,
// 1 im) of complex input n, so the 8 halves a lane holds in one 16-wide K step are the
// (re, im) pairs of inputs n = 8q + 4(l/32) + 0..3 -- exactly four stored four-byte
// complex values, used as they are loaded.  A 32-row output block holds 16 complex
// outputs: rows 0..15 their real parts, rows 16..31 their imaginary parts, so that
// after a product lane l holds the real and imaginary part of the same 8 outputs:
//   out k' = 4(l/32) + r      : (D[r],     D[8 + r])
//   out k' = 8 + 4(l/32) + r  : (D[4 + r], D[12 + r])     r = 0..3.
// The constant DFT-matrix operands are built on the host in FP64 (mfma_tables.cpp) and
// stored as 64 lanes x 16 bytes per operand.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "nlos_internal.hpp"

namespace nlos {

typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 mf_b8 __attribute__((ext_vector_type(8)));
typedef float mf_acc __attribute__((ext_vector_type(16)));
typedef unsigned int mf_u4 __attribute__((ext_vector_type(4)));
typedef _Float16 mf_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 mf_bf2 __attribute__((ext_vector_type(2)));

template <int SP>
struct Mfma;

template <>
struct Mfma<SP_F16> {
  static __device__ __forceinline__ mf_acc mma(mf_u4 a, mf_u4 b, mf_acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(mf_h8, a), __builtin_bit_cast(mf_h8, b), c, 0,
                                                  0, 0);
  }
  // (re, im) -> one dword, round to nearest even
  static __device__ __forceinline__ unsigned int pack(float re, float im) {
    const mf_h2 h = {(_Float16)re, (_Float16)im};
    return __builtin_bit_cast(unsigned int, h);
  }
  static __device__ __forceinline__ float2 unpack(unsigned int u) {
    const mf_h2 h = __builtin_bit_cast(mf_h2, u);
    return make_float2((float)h.x, (float)h.y);
  }
};

template <>
struct Mfma<SP_BF16> {
  static __device__ __forceinline__ mf_acc mma(mf_u4 a, mf_u4 b, mf_acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(mf_b8, a), __builtin_bit_cast(mf_b8, b), c,
                                                   0, 0, 0);
  }
  static __device__ __forceinline__ unsigned int pack(float re, float im) {
    const mf_bf2 h = {(__bf16)re, (__bf16)im};
    return __builtin_bit_cast(unsigned int, h);
  }
  static __device__ __forceinline__ float2 unpack(unsigned int u) {
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  }
};

// Output k' (0..15) of a 16-output block held by this lane as slot j (0..7):
// j < 4: k' = 4 hl + j; j >= 4: k' = 8 + 4 hl + (j - 4), with (re, im) = (D[j], D[j + 8]).
__device__ __forceinline__ int mf_out_index(int j, int hl) { return (j < 4 ? 0 : 8) + 4 * hl + (j & 3); }
__device__ __forceinline__ float2 mf_out(const mf_acc& d, int j) { return make_float2(d[j], d[j + 8]); }

// complex multiply in FP32 (w conjugated when CONJ)
template <bool CONJ>
__device__ __forceinline__ float2 mf_cmul(float2 a, float2 w) {
  const float wy = CONJ ? -w.y : w.y;
  return make_float2(fmaf(a.x, w.x, -a.y * wy), fmaf(a.x, wy, a.y * w.x));
}

}  // namespace nlos

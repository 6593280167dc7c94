// Storage precision of the complex intermediates: FP32 (float2), FP16 (two binary16)
// or BF16 (two bfloat16), four bytes per complex value in the reduced forms.
//
// FP16 values are stored times a power of two 2^e fixed per intermediate (chosen on the
// device from a bound on the intermediate's magnitude, so the largest stored value stays
// below 2^14) and multiplied by 2^-e when read: exact scalings, so only the FP16
// rounding of each store remains.  BF16 has FP32's exponent range and is stored as is.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "nlos_internal.hpp"

namespace nlos {

template <int SP>
struct Stor;

// ld(p, i) loads and converts; readers that load many values under conditions use
// raw(p, i) (the stored bits, R) inside the condition and cvt(R) after all loads, so
// that the loads stay in flight together instead of each waiting for its conversion.
// The four-byte forms hold only f-k volumes, which every pass streams once: their
// loads and stores are non-temporal.
template <>
struct Stor<SP_F32> {
  using T = float2;
  using R = float2;
  static __device__ __forceinline__ R zero() { return make_float2(0.f, 0.f); }
  static __device__ __forceinline__ R raw(const T* p, long long i) { return p[i]; }
  static __device__ __forceinline__ float2 cvt(R r) { return r; }
  static __device__ __forceinline__ float2 ld(const T* p, long long i) { return p[i]; }
  static __device__ __forceinline__ void st(T* p, long long i, float2 v) { p[i] = v; }
  // two consecutive values (i even: one 16-byte store)
  static __device__ __forceinline__ void st2(T* p, long long i, float2 a, float2 b) {
    *reinterpret_cast<float4*>(p + i) = make_float4(a.x, a.y, b.x, b.y);
  }
};

typedef _Float16 nlos_h2 __attribute__((ext_vector_type(2)));
typedef __bf16 nlos_bf2 __attribute__((ext_vector_type(2)));

template <>
struct Stor<SP_F16> {
  using T = __half2;
  using R = unsigned int;
  static __device__ __forceinline__ R zero() { return 0u; }
  static __device__ __forceinline__ R raw(const T* p, long long i) {
    return __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p) + i);
  }
  static __device__ __forceinline__ float2 cvt(R r) {
    const nlos_h2 h = __builtin_bit_cast(nlos_h2, r);
    return make_float2((float)h.x, (float)h.y);
  }
  static __device__ __forceinline__ float2 ld(const T* p, long long i) { return cvt(raw(p, i)); }
  static __device__ __forceinline__ unsigned int pack(float2 v) {
    const nlos_h2 h = {(_Float16)v.x, (_Float16)v.y};  // round to nearest even
    return __builtin_bit_cast(unsigned int, h);
  }
  static __device__ __forceinline__ void st(T* p, long long i, float2 v) {
    __builtin_nontemporal_store(pack(v), reinterpret_cast<unsigned int*>(p) + i);
  }
  // two consecutive values (i even: one 8-byte store)
  static __device__ __forceinline__ void st2(T* p, long long i, float2 a, float2 b) {
    typedef unsigned int u2v __attribute__((ext_vector_type(2)));
    const u2v w = {pack(a), pack(b)};
    __builtin_nontemporal_store(w, reinterpret_cast<u2v*>(p + i));
  }
};

template <>
struct Stor<SP_BF16> {
  using T = __hip_bfloat162;
  using R = unsigned int;
  static __device__ __forceinline__ R zero() { return 0u; }
  static __device__ __forceinline__ R raw(const T* p, long long i) {
    return __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p) + i);
  }
  // a bfloat16 is the upper half of the float with the same bits
  static __device__ __forceinline__ float2 cvt(R r) {
    return make_float2(__uint_as_float(r << 16), __uint_as_float(r & 0xffff0000u));
  }
  static __device__ __forceinline__ float2 ld(const T* p, long long i) { return cvt(raw(p, i)); }
  // round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
  static __device__ __forceinline__ unsigned int pack(float2 v) {
    const nlos_bf2 h = {(__bf16)v.x, (__bf16)v.y};
    return __builtin_bit_cast(unsigned int, h);
  }
  static __device__ __forceinline__ void st(T* p, long long i, float2 v) {
    __builtin_nontemporal_store(pack(v), reinterpret_cast<unsigned int*>(p) + i);
  }
  // two consecutive values (i even: one 8-byte store)
  static __device__ __forceinline__ void st2(T* p, long long i, float2 a, float2 b) {
    typedef unsigned int u2v __attribute__((ext_vector_type(2)));
    const u2v w = {pack(a), pack(b)};
    __builtin_nontemporal_store(w, reinterpret_cast<u2v*>(p + i));
  }
};

__device__ __forceinline__ float2 ldexp2(float2 v, int e) {
  return make_float2(ldexpf(v.x, e), ldexpf(v.y, e));
}

}  // namespace nlos

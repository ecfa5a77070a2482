// Element types, conversions and the MFMA step shared by the network kernels (gfx950).
//
// Every operand fragment is 16 bytes per lane.  With float the fragment holds four
// channels and feeds four v_mfma_f32_16x16x4_f32 (K = 4 each); with float16 or
// bfloat16 it holds eight channels and feeds one v_mfma_f32_16x16x32_{f16,bf16}.  In
// both cases a 16-channel (float) or 32-channel (16-bit) group is split over the four
// lane quarters q = lane / 16, quarter q taking the group's channels
// [q * KG/4, (q+1) * KG/4).  A (weights) and B (activations) use the same split, so
// the K pairing is consistent; the output D[i][j] sits in lane j + 16 * (i / 4),
// item i % 4, for all three instructions.
#pragma once
#include "nv_device.h"

namespace nv {

typedef _Float16 f16;
typedef __bf16 bf16;
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mma;

template <>
struct Mma<float> {
  static constexpr int KG = 16;   // channels per fragment group
  __device__ static __forceinline__ f32x4 step(u32x4 a, u32x4 b, f32x4 acc) {
    const f32x4 fa = __builtin_bit_cast(f32x4, a), fb = __builtin_bit_cast(f32x4, b);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[kk], fb[kk], acc, 0, 0, 0);
    return acc;
  }
};

template <>
struct Mma<f16> {
  static constexpr int KG = 32;
  __device__ static __forceinline__ f32x4 step(u32x4 a, u32x4 b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
  }
};

template <>
struct Mma<bf16> {
  static constexpr int KG = 32;
  __device__ static __forceinline__ f32x4 step(u32x4 a, u32x4 b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  }
};

__device__ __forceinline__ u32x4 ldu4(const void* p) { return *reinterpret_cast<const u32x4*>(p); }
__device__ __forceinline__ void stu4(void* p, u32x4 v) { *reinterpret_cast<u32x4*>(p) = v; }

// Four consecutive elements <-> four floats.
template <typename T>
__device__ __forceinline__ f32x4 load4f(const T* p);
template <>
__device__ __forceinline__ f32x4 load4f<float>(const float* p) { return ld4(p); }
template <>
__device__ __forceinline__ f32x4 load4f<f16>(const f16* p) {
  const f16x4 v = *reinterpret_cast<const f16x4*>(p);
  return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
template <>
__device__ __forceinline__ f32x4 load4f<bf16>(const bf16* p) {
  const bf16x4 v = *reinterpret_cast<const bf16x4*>(p);
  return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}

template <typename T>
__device__ __forceinline__ void store4f(T* p, f32x4 v);
template <>
__device__ __forceinline__ void store4f<float>(float* p, f32x4 v) { st4(p, v); }
template <>
__device__ __forceinline__ void store4f<f16>(f16* p, f32x4 v) {
  *reinterpret_cast<f16x4*>(p) = f16x4{(f16)v[0], (f16)v[1], (f16)v[2], (f16)v[3]};
}
template <>
__device__ __forceinline__ void store4f<bf16>(bf16* p, f32x4 v) {
  *reinterpret_cast<bf16x4*>(p) = bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
}

// Eight consecutive elements of type TIN, converted, stored as eight TC at q (LDS).
template <typename TIN, typename TC>
__device__ __forceinline__ void copy8(TC* q, const TIN* p) {
  f32x4 lo = load4f<TIN>(p), hi = load4f<TIN>(p + 4);
  store4f<TC>(q, lo);
  store4f<TC>(q + 4, hi);
}
template <>
__device__ __forceinline__ void copy8<f16, f16>(f16* q, const f16* p) { stu4(q, ldu4(p)); }
template <>
__device__ __forceinline__ void copy8<bf16, bf16>(bf16* q, const bf16* p) { stu4(q, ldu4(p)); }

template <typename TC>
__device__ __forceinline__ void zero8(TC* q) {
  store4f<TC>(q, zero4());
  store4f<TC>(q + 4, zero4());
}

__device__ __forceinline__ f32x4 lrelu4(f32x4 v) {
  return f32x4{lrelu(v[0]), lrelu(v[1]), lrelu(v[2]), lrelu(v[3])};
}

}  // namespace nv

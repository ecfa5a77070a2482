// Element types, conversions and the MFMA step shared by the network kernels (gfx950).
//
// With float the operand fragment is 16 bytes per lane holding four channels and feeds
// four v_mfma_f32_16x16x4_f32 (K = 4 each); with float16 or bfloat16 it is 16 bytes
// holding eight channels and feeds one v_mfma_f32_16x16x32_{f16,bf16}; with FP8 e4m3
// it is 32 bytes holding 32 channels and feeds one v_mfma_scale_f32_16x16x128_f8f6f4
// (unit block scales: the per-channel scales are applied in the epilogues).  A group
// of KG = 16 / 32 / 128 reduction indices is split over the four lane quarters
// q = lane / 16, quarter q taking indices [q * KG/4, (q+1) * KG/4).  A (weights) and
// B (activations) use the same split, so the K pairing is consistent; the output
// D[i][j] sits in lane j + 16 * (i / 4), item i % 4, for all four instructions.
#pragma once
#include <type_traits>

#include "nv_device.h"

namespace nv {

typedef _Float16 f16;
typedef __bf16 bf16;
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// One OCP FP8 e4m3 value (bias 7, largest finite 448, no infinities).
struct f8 {
  uint8_t bits;
};
constexpr float kF8Max = 448.0f;

__device__ __forceinline__ u32x4 ldu4(const void* p) { return *reinterpret_cast<const u32x4*>(p); }
__device__ __forceinline__ void stu4(void* p, u32x4 v) { *reinterpret_cast<u32x4*>(p) = v; }
__device__ __forceinline__ u32x8 ldu8(const void* p) {
  const u32x4 lo = ldu4(p), hi = ldu4(static_cast<const uint8_t*>(p) + 16);
  return u32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

template <typename T>
struct Mma;

template <>
struct Mma<float> {
  static constexpr int KG = 16;   // channels per fragment group
  typedef u32x4 Frag;
  __device__ static __forceinline__ Frag ld(const void* p) { return ldu4(p); }
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
  typedef u32x4 Frag;
  __device__ static __forceinline__ Frag ld(const void* p) { return ldu4(p); }
  __device__ static __forceinline__ f32x4 step(u32x4 a, u32x4 b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                   __builtin_bit_cast(f16x8, b), acc, 0, 0, 0);
  }
};

template <>
struct Mma<bf16> {
  static constexpr int KG = 32;
  typedef u32x4 Frag;
  __device__ static __forceinline__ Frag ld(const void* p) { return ldu4(p); }
  __device__ static __forceinline__ f32x4 step(u32x4 a, u32x4 b, f32x4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
  }
};

template <>
struct Mma<f8> {
  static constexpr int KG = 128;
  typedef u32x8 Frag;
  __device__ static __forceinline__ Frag ld(const void* p) { return ldu8(p); }
  __device__ static __forceinline__ f32x4 step(u32x8 a, u32x8 b, f32x4 acc) {
    // formats 0 / 0 = e4m3 for A and B; block scales 127 = 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(__builtin_bit_cast(i32x8, a),
                                                             __builtin_bit_cast(i32x8, b), acc, 0, 0, 0, 127,
                                                             0, 127);
  }
};

// Four floats -> four e4m3 bytes (round to nearest even).  The inputs are clamped to
// the finite range first, so nothing converts to NaN.
__device__ __forceinline__ uint32_t f8x4_pack(f32x4 v) {
  f32x4 c;
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = fminf(fmaxf(v[i], -kF8Max), kF8Max);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
  return (uint32_t)w;
}

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

// Eight consecutive elements -> two float vectors (one 16-byte load for 16-bit types).
template <typename T>
__device__ __forceinline__ void load8f(const T* p, f32x4& lo, f32x4& hi) {
  lo = load4f<T>(p);
  hi = load4f<T>(p + 4);
}
template <>
__device__ __forceinline__ void load8f<f16>(const f16* p, f32x4& lo, f32x4& hi) {
  const f16x8 v = *reinterpret_cast<const f16x8*>(p);
  lo = f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  hi = f32x4{(float)v[4], (float)v[5], (float)v[6], (float)v[7]};
}
template <>
__device__ __forceinline__ void load8f<bf16>(const bf16* p, f32x4& lo, f32x4& hi) {
  const bf16x8 v = *reinterpret_cast<const bf16x8*>(p);
  lo = f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  hi = f32x4{(float)v[4], (float)v[5], (float)v[6], (float)v[7]};
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
template <>
__device__ __forceinline__ void store4f<f8>(f8* p, f32x4 v) {
  *reinterpret_cast<uint32_t*>(p) = f8x4_pack(v);
}

// Eight values stored as eight consecutive TC with one store where they fit 16 bytes.
template <typename TC>
__device__ __forceinline__ void store8f(TC* p, f32x4 lo, f32x4 hi) {
  store4f<TC>(p, lo);
  store4f<TC>(p + 4, hi);
}
template <>
__device__ __forceinline__ void store8f<f16>(f16* p, f32x4 lo, f32x4 hi) {
  *reinterpret_cast<f16x8*>(p) = f16x8{(f16)lo[0], (f16)lo[1], (f16)lo[2], (f16)lo[3],
                                       (f16)hi[0], (f16)hi[1], (f16)hi[2], (f16)hi[3]};
}
template <>
__device__ __forceinline__ void store8f<bf16>(bf16* p, f32x4 lo, f32x4 hi) {
  *reinterpret_cast<bf16x8*>(p) = bf16x8{(bf16)lo[0], (bf16)lo[1], (bf16)lo[2], (bf16)lo[3],
                                         (bf16)hi[0], (bf16)hi[1], (bf16)hi[2], (bf16)hi[3]};
}
template <>
__device__ __forceinline__ void store8f<f8>(f8* p, f32x4 lo, f32x4 hi) {
  *reinterpret_cast<u32x2*>(p) = u32x2{f8x4_pack(lo), f8x4_pack(hi)};
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

// Eight consecutive elements held as loaded (so that a thread can issue all of its
// staging loads before the first LDS store), then converted to the LDS type.
template <typename T>
struct Raw8 {
  u32x4 v;                                  // 16-bit types: 8 x 2 bytes
  __device__ __forceinline__ void load(const T* p) { v = ldu4(p); }
  __device__ __forceinline__ void zero() { v = u32x4{0u, 0u, 0u, 0u}; }
  __device__ __forceinline__ void to_f32(f32x4& lo, f32x4& hi) const {
    typedef T T8 __attribute__((ext_vector_type(8)));
    const T8 e = __builtin_bit_cast(T8, v);
    lo = f32x4{(float)e[0], (float)e[1], (float)e[2], (float)e[3]};
    hi = f32x4{(float)e[4], (float)e[5], (float)e[6], (float)e[7]};
  }
};
template <>
struct Raw8<float> {
  f32x4 lo, hi;
  __device__ __forceinline__ void load(const float* p) {
    lo = ld4(p);
    hi = ld4(p + 4);
  }
  __device__ __forceinline__ void zero() { lo = hi = zero4(); }
  __device__ __forceinline__ void to_f32(f32x4& a, f32x4& b) const {
    a = lo;
    b = hi;
  }
};

template <typename TIN, typename TC>
__device__ __forceinline__ void raw8_store(TC* q, const Raw8<TIN>& r) {
  if constexpr (std::is_same<TIN, TC>::value && !std::is_same<TIN, float>::value) {
    stu4(q, r.v);
  } else {
    f32x4 lo, hi;
    r.to_f32(lo, hi);
    store4f<TC>(q, lo);
    store4f<TC>(q + 4, hi);
  }
}

// Eight floats staged as float16: part 0 the rounded values, part 1 the float16 of
// what the rounding left out (x = hi + lo to about 22 bits).
__device__ __forceinline__ void copy8_split(f16* q, const Raw8<float>& r, int part) {
  f32x4 v[2] = {r.lo, r.hi};
  f16x8 o;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const f16 hi = (f16)v[h][i];
      o[4 * h + i] = part == 0 ? hi : (f16)(v[h][i] - (float)hi);
    }
  *reinterpret_cast<f16x8*>(q) = o;
}

template <typename TC>
__device__ __forceinline__ void zero8(TC* q) {
  store4f<TC>(q, zero4());
  store4f<TC>(q + 4, zero4());
}

__device__ __forceinline__ f32x4 lrelu4(f32x4 v) {
  return f32x4{lrelu(v[0]), lrelu(v[1]), lrelu(v[2]), lrelu(v[3])};
}

}  // namespace nv

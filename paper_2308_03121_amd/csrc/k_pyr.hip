// Feature-pyramid kernels (gfx950): the 2x2 mean pool that starts a pyramid level, and
// the x2 bilinear resize of a coarser level added into a finer one (the cascade of the
// aligned features and of the offsets).  Both are elementwise over NHWC maps and bound
// by HBM traffic: each thread moves 16 bytes per map access (four channels of a float
// map, eight of a 16-bit one), consecutive threads take consecutive channel vectors of
// a pixel, so every wave reads and writes whole contiguous pixels.
#include <type_traits>

#include "nv_internal.h"
#include "nv_mma.h"

namespace nv {
namespace {

// 16 bytes of a map as floats (E = 4 for float, 8 for 16-bit types) and back.
template <typename T>
struct Vec16 {
  static constexpr int E = 16 / (int)sizeof(T);
  float v[E];
  __device__ __forceinline__ void load(const T* p) {
    if constexpr (std::is_same<T, float>::value) {
      const f32x4 a = ld4(p);
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = a[i];
    } else {
      f32x4 lo, hi;
      load8f<T>(p, lo, hi);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = lo[i];
        v[4 + i] = hi[i];
      }
    }
  }
  __device__ __forceinline__ void store(T* p) const {
    if constexpr (std::is_same<T, float>::value) {
      st4(p, f32x4{v[0], v[1], v[2], v[3]});
    } else {
      store8f<T>(p, f32x4{v[0], v[1], v[2], v[3]}, f32x4{v[4], v[5], v[6], v[7]});
    }
  }
};

// dst (H2 x W2 x C) = mean of the 2x2 blocks of src (2 H2 x 2 W2 x C), summed as
// (top pair + bottom pair) / 4 in float and rounded to T once.
template <typename T>
__global__ __launch_bounds__(256) void k_pool2(const T* __restrict__ src, T* __restrict__ dst, int H2, int W2,
                                               int C) {
  using V = Vec16<T>;
  const int nv = C / V::E;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)H2 * W2 * nv) return;
  const int cv = (int)(idx % nv);
  const int64_t p = idx / nv;
  const int y = (int)(p / W2), x = (int)(p % W2);
  const int W = 2 * W2;
  const T* s0 = src + ((int64_t)(2 * y) * W + 2 * x) * C + cv * V::E;
  const T* s1 = s0 + (int64_t)W * C;
  V a, b, c, d, o;
  a.load(s0);
  b.load(s0 + C);
  c.load(s1);
  d.load(s1 + C);
#pragma unroll
  for (int i = 0; i < V::E; ++i) o.v[i] = ((a.v[i] + b.v[i]) + (c.v[i] + d.v[i])) * 0.25f;
  o.store(dst + p * C + cv * V::E);
}

// dst[y][x][c] += scale * up2(src)[y][x][c] for c < nch, dst H x W (channel stride ldd),
// src H/2 x W/2 (channel stride lds).  up2: output row 2i + r takes 3/4 of row i and 1/4
// of row i - 1 (r = 0) or i + 1 (r = 1), clamped at the edges; the same along columns.
template <typename T>
__global__ __launch_bounds__(256) void k_up2_add(T* __restrict__ dst, int ldd, const T* __restrict__ src, int lds,
                                                 int H, int W, int nch, float scale) {
  using V = Vec16<T>;
  const int nv = nch / V::E;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)H * W * nv) return;
  const int cv = (int)(idx % nv);
  const int64_t p = idx / nv;
  const int y = (int)(p / W), x = (int)(p % W);
  const int Hc = H / 2, Wc = W / 2;
  const int i = y >> 1, j = x >> 1;
  const int in = min(max((y & 1) ? i + 1 : i - 1, 0), Hc - 1);
  const int jn = min(max((x & 1) ? j + 1 : j - 1, 0), Wc - 1);
  const T* r0 = src + (int64_t)i * Wc * lds + cv * V::E;
  const T* r1 = src + (int64_t)in * Wc * lds + cv * V::E;
  V a, b, c, d, o;
  a.load(r0 + (int64_t)j * lds);
  b.load(r0 + (int64_t)jn * lds);
  c.load(r1 + (int64_t)j * lds);
  d.load(r1 + (int64_t)jn * lds);
  T* q = dst + p * ldd + cv * V::E;
  o.load(q);
#pragma unroll
  for (int e = 0; e < V::E; ++e) {
    const float u = 0.75f * (0.75f * a.v[e] + 0.25f * b.v[e]) + 0.25f * (0.75f * c.v[e] + 0.25f * d.v[e]);
    o.v[e] += scale * u;
  }
  o.store(q);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_pool2(int t, const void* src, void* dst, int H2, int W2, int C, hipStream_t s) {
  if (H2 <= 0 || W2 <= 0 || C % 8 != 0) return hipErrorInvalidValue;
  const int64_t n = (int64_t)H2 * W2 * C;
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(k_pool2<float>, dim3(blocks_for(n / 4)), dim3(256), 0, s, static_cast<const float*>(src),
                         static_cast<float*>(dst), H2, W2, C);
      break;
    case DT_F16:
      hipLaunchKernelGGL(k_pool2<f16>, dim3(blocks_for(n / 8)), dim3(256), 0, s, static_cast<const f16*>(src),
                         static_cast<f16*>(dst), H2, W2, C);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_pool2<bf16>, dim3(blocks_for(n / 8)), dim3(256), 0, s, static_cast<const bf16*>(src),
                         static_cast<bf16*>(dst), H2, W2, C);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_up2_add(int t, void* dst, int ldd, const void* src, int lds, int H, int W, int nch, float scale,
                          hipStream_t s) {
  const int e = t == DT_F32 ? 4 : 8;   // channels per 16-byte vector
  if (H <= 0 || W <= 0 || (H | W) & 1 || nch % e != 0 || ldd % e != 0 || lds % e != 0 || nch > ldd || nch > lds)
    return hipErrorInvalidValue;
  const int64_t n = (int64_t)H * W * nch;
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(k_up2_add<float>, dim3(blocks_for(n / 4)), dim3(256), 0, s, static_cast<float*>(dst), ldd,
                         static_cast<const float*>(src), lds, H, W, nch, scale);
      break;
    case DT_F16:
      hipLaunchKernelGGL(k_up2_add<f16>, dim3(blocks_for(n / 8)), dim3(256), 0, s, static_cast<f16*>(dst), ldd,
                         static_cast<const f16*>(src), lds, H, W, nch, scale);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(k_up2_add<bf16>, dim3(blocks_for(n / 8)), dim3(256), 0, s, static_cast<bf16*>(dst), ldd,
                         static_cast<const bf16*>(src), lds, H, W, nch, scale);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace nv

// Device-side helpers shared by the gfx950 kernels of the enhancement library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nv {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr float kLreluSlope = 0.1f;

// Width in pixels of the network kernels' output tiles (one MFMA column block).
constexpr int kTW = 16;

// BT.709 luma weights; every derived coefficient is formed in double and rounded once.
constexpr double kKr = 0.2126;
constexpr double kKb = 0.0722;
constexpr double kKg = 1.0 - kKr - kKb;

__device__ __forceinline__ float lrelu(float v) { return v >= 0.0f ? v : kLreluSlope * v; }

__device__ __forceinline__ float sigmoidf(float v) { return 1.0f / (1.0f + __expf(-v)); }

__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }

__device__ __forceinline__ void st4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.0f, 0.0f, 0.0f, 0.0f}; }

// One MFMA: D(16x16, fp32) += A(16x4) * B(4x16).  Operand lane layout (wave64):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane j + 16*(i/4), item i%4.
__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// Linear block index remapped so that each of the 8 XCDs (which receive workgroups
// round-robin) processes one contiguous range of tiles; neighbouring tiles then share
// their halo rows in the same L2.  Identity when the grid does not split evenly.
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  if ((nblk & 7) != 0) return bid;
  const int per = nblk >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Smallest j with jobs[j+1].item_begin > item (jobs sorted by item_begin, njobs >= 1).
template <class J>
__device__ __forceinline__ int find_job(const J* jobs, int njobs, int item) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item_begin <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace nv

// CPU simulation of the HIP device and runtime for the library's kernels (test build
// only; see tests/test_cpusim.py).  The kernels and the host runtime are compiled as
// ordinary host C++ against this header: "device" memory is host memory, every
// work-item of a workgroup runs as a fiber on one OS thread, __syncthreads() and the
// wave-wide operations (MFMA, lane shuffles, readfirstlane) are rendezvous points, and
// __shared__ arrays are function statics.  Workgroups run one after another.  A
// barrier that some live work-items never reach, or a wave operation that not every
// live lane of the wave joins, is reported as a hang instead of blocking.  The product
// is always built with hipcc against the real HIP runtime.
#pragma once
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <utility>

// ------------------------------------------------------------------ runtime ----
typedef enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidConfiguration = 9,
  hipErrorNotSupported = 801,
} hipError_t;

typedef enum {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
} hipMemcpyKind;

typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1, hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;
typedef enum { hipDeviceAttributeMaxSharedMemoryPerBlock = 74 } hipDeviceAttribute_t;

enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
enum { hipStreamDefault = 0, hipStreamNonBlocking = 1 };
enum { hipHostMallocDefault = 0 };

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph* hipGraph_t;
typedef struct hipGraphExec* hipGraphExec_t;

const char* hipGetErrorString(hipError_t e);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                             size_t height, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemset(void* p, int v, size_t bytes);
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t s);
hipError_t hipDeviceSynchronize(void);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipGetLastError(void);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, void* a, void* b, size_t c);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(x) (reinterpret_cast<const void*>(&(x)))
#define __align__(n) __attribute__((aligned(n)))

// -------------------------------------------------------------- device side ----
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct nvsim_uint3 {
  unsigned x, y, z;
};

namespace nvsim {
extern nvsim_uint3 g_thread, g_block;
extern dim3 g_block_dim, g_grid_dim;

typedef float f32x4_ __attribute__((ext_vector_type(4)));
typedef float f32x16_ __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8_ __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_ __attribute__((ext_vector_type(8)));
typedef int i32x8_ __attribute__((ext_vector_type(8)));

void syncthreads();
f32x4_ mfma_f32_16x16x4f32(float a, float b, f32x4_ c, int, int, int);
f32x4_ mfma_f32_16x16x32_f16(f16x8_ a, f16x8_ b, f32x4_ c, int, int, int);
f32x4_ mfma_f32_16x16x32_bf16(bf16x8_ a, bf16x8_ b, f32x4_ c, int, int, int);
f32x16_ mfma_f32_32x32x16_f16(f16x8_ a, f16x8_ b, f32x16_ c, int, int, int);
f32x16_ mfma_f32_32x32x16_bf16(bf16x8_ a, bf16x8_ b, f32x16_ c, int, int, int);
f32x4_ mfma_scale_f32_16x16x128_f8f6f4(i32x8_ a, i32x8_ b, f32x4_ c, int fa, int fb, int, int sa, int, int sb);
int cvt_pk_fp8_f32(float a, float b, int old, bool hi);
uint64_t shfl_xor_bits(uint64_t v, int mask, int width);
int readfirstlane(int v);

// one kernel launch: run body once per work-item of every workgroup (or record it
// when the stream is being captured)
void launch(dim3 grid, dim3 block, hipStream_t s, std::function<void()> body);
template <class F, class... A>
void launch_args(dim3 grid, dim3 block, hipStream_t s, F f, A... a) {
  launch(grid, block, s, [f, a...]() { f(a...); });
}

template <class T>
T shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "scalar lane values");
  uint64_t b = 0;
  memcpy(&b, &v, sizeof(T));
  b = shfl_xor_bits(b, mask, width);
  T r;
  memcpy(&r, &b, sizeof(T));
  return r;
}
}  // namespace nvsim

#define threadIdx (::nvsim::g_thread)
#define blockIdx (::nvsim::g_block)
#define blockDim (::nvsim::g_block_dim)
#define gridDim (::nvsim::g_grid_dim)

#define __syncthreads() ::nvsim::syncthreads()
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_mfma_f32_16x16x4f32 ::nvsim::mfma_f32_16x16x4f32
#define __builtin_amdgcn_mfma_f32_16x16x32_f16 ::nvsim::mfma_f32_16x16x32_f16
#define __builtin_amdgcn_mfma_f32_16x16x32_bf16 ::nvsim::mfma_f32_16x16x32_bf16
#define __builtin_amdgcn_mfma_f32_32x32x16_f16 ::nvsim::mfma_f32_32x32x16_f16
#define __builtin_amdgcn_mfma_f32_32x32x16_bf16 ::nvsim::mfma_f32_32x32x16_bf16
#define __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4 ::nvsim::mfma_scale_f32_16x16x128_f8f6f4
#define __builtin_amdgcn_cvt_pk_fp8_f32 ::nvsim::cvt_pk_fp8_f32
#define __builtin_amdgcn_readfirstlane ::nvsim::readfirstlane
#define __shfl_xor ::nvsim::shfl_xor
#define hipLaunchKernelGGL(K, G, B, M, S, ...) \
  ::nvsim::launch_args(dim3(G), dim3(B), (S), [](auto... a_) { K(a_...); }, __VA_ARGS__)

inline float __expf(float x) { return expf(x); }
inline unsigned __float_as_uint(float x) {
  unsigned u;
  memcpy(&u, &x, 4);
  return u;
}
inline float __uint_as_float(unsigned u) {
  float x;
  memcpy(&x, &u, 4);
  return x;
}
// workgroups run one at a time on one OS thread, so plain read-modify-writes are atomic
template <class T>
inline T atomicAdd(T* p, T v) {
  const T o = *p;
  *p = o + v;
  return o;
}
template <class T>
inline T atomicMax(T* p, T v) {
  const T o = *p;
  if (v > o) *p = v;
  return o;
}
template <class T>
inline T min(T a, T b) {
  return b < a ? b : a;
}
template <class T>
inline T max(T a, T b) {
  return a < b ? b : a;
}

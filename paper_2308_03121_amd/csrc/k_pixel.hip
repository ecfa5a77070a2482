// Pixel-format and scene-change kernels (gfx950).
//
// Unpack: Y'CbCr codes -> planar float32 R'G'B' with alignment padding.
// Pack:   planar float32 R'G'B' -> Y'CbCr codes with crop.
// Scene:  integer SAD and 64-bin histogram distance, and the cut decision.
// All three are HBM-bound streaming kernels; each thread owns a small run of
// adjacent pixels so that row accesses coalesce.  Every stage has a single-frame
// launch and a batched, persistent launch over a device table of frames (possibly of
// different sizes and formats).
#include "nv_device.h"
#include "nv_internal.h"

namespace nv {

namespace {

// Luma weights (Kr, Kb) of ITU-R BT.601, BT.709 and BT.2020 (non-constant luminance).
void luma_weights(int matrix, double& kr, double& kb) {
  if (matrix == 601) {
    kr = 0.299;
    kb = 0.114;
  } else if (matrix == 2020) {
    kr = 0.2627;
    kb = 0.0593;
  } else {
    kr = kKr;
    kb = kKb;
  }
}

// Code scale and offset of luma and chroma: limited range 219 / 16 and 224 / 128 times
// 2^(b-8); full range 2^b - 1 / 0 and 2^b - 1 / 2^(b-1).
void code_range(int bits, int full, double& ys, double& yo, double& cs, double& co) {
  if (full) {
    ys = cs = double((1 << bits) - 1);
    yo = 0.0;
    co = double(1 << (bits - 1));
  } else {
    const double s = double(1 << (bits - 8));
    ys = 219.0 * s;
    yo = 16.0 * s;
    cs = 224.0 * s;
    co = 128.0 * s;
  }
}

}  // namespace

Inv make_inv(int bits, int matrix, int full) {
  double kr, kb, ys, yo, cs, co;
  luma_weights(matrix, kr, kb);
  code_range(bits, full, ys, yo, cs, co);
  const double kg = 1.0 - kr - kb;
  Inv m;
  m.ys = float(1.0 / ys);
  m.yo = float(yo);
  m.cs = float(1.0 / cs);
  m.co = float(co);
  m.rcr = float(2.0 * (1.0 - kr));
  m.bcb = float(2.0 * (1.0 - kb));
  m.gcb = float(2.0 * kb * (1.0 - kb) / kg);
  m.gcr = float(2.0 * kr * (1.0 - kr) / kg);
  return m;
}

Fwd make_fwd(int bits, int matrix, int full) {
  double kr, kb, ys, yo, cs, co;
  luma_weights(matrix, kr, kb);
  code_range(bits, full, ys, yo, cs, co);
  Fwd m;
  m.kr = float(kr);
  m.kg = float(1.0 - kr - kb);
  m.kb = float(kb);
  m.cbs = float(1.0 / (2.0 * (1.0 - kb)));
  m.crs = float(1.0 / (2.0 * (1.0 - kr)));
  m.ys = float(ys);
  m.yo = float(yo);
  m.cs = float(cs);
  m.co = float(co);
  m.maxc = float((1 << bits) - 1);
  return m;
}

namespace {

template <int BITS>
struct Code;
template <>
struct Code<8> {
  static __device__ __forceinline__ float get(const void* p, int64_t pitch, int y, int x) {
    return (float)reinterpret_cast<const uint8_t*>(static_cast<const char*>(p) + y * pitch)[x];
  }
  static __device__ __forceinline__ void put(void* p, int64_t pitch, int y, int x, int v) {
    reinterpret_cast<uint8_t*>(static_cast<char*>(p) + y * pitch)[x] = (uint8_t)v;
  }
};
template <>
struct Code<10> {
  static __device__ __forceinline__ float get(const void* p, int64_t pitch, int y, int x) {
    return (float)(reinterpret_cast<const uint16_t*>(static_cast<const char*>(p) + y * pitch)[x] &
                   0x3FFu);
  }
  static __device__ __forceinline__ void put(void* p, int64_t pitch, int y, int x, int v) {
    reinterpret_cast<uint16_t*>(static_cast<char*>(p) + y * pitch)[x] = (uint16_t)v;
  }
};

// N consecutive codes of row y starting at column x0 (N = 4 or 8), columns clamped to
// w - 1.  A run inside the row whose address is aligned to its size is one vector load.
template <int BITS, int N>
__device__ __forceinline__ void code_run(const void* base, int64_t pitch, int y, int x0, int w, float (&v)[N]) {
  constexpr int SB = BITS == 8 ? 1 : 2;      // bytes per sample
  constexpr int VB = N * SB;                 // 4, 8 or 16 bytes
  constexpr uint32_t mask = BITS == 8 ? 0xFFu : 0x3FFu;
  const char* row = static_cast<const char*>(base) + y * pitch;
  const char* at = row + (size_t)x0 * SB;
  if (x0 + N <= w && (reinterpret_cast<uintptr_t>(at) & (VB - 1)) == 0) {
    uint32_t wd[VB / 4];
    if constexpr (VB == 4) {
      wd[0] = *reinterpret_cast<const uint32_t*>(at);
    } else if constexpr (VB == 8) {
      const u32x2 t = *reinterpret_cast<const u32x2*>(at);
      wd[0] = t[0];
      wd[1] = t[1];
    } else {
      const u32x4 t = *reinterpret_cast<const u32x4*>(at);
      wd[0] = t[0];
      wd[1] = t[1];
      wd[2] = t[2];
      wd[3] = t[3];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      constexpr int PER = 4 / SB;            // samples per 32-bit word
      v[k] = (float)((wd[k / PER] >> (8 * SB * (k % PER))) & mask);
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = Code<BITS>::get(base, pitch, y, min(x0 + k, w - 1));
  }
}

// N codes written to row y from column x0 (all inside the row): one vector store when
// aligned, else one store per sample.
template <int BITS, int N>
__device__ __forceinline__ void code_store(void* base, int64_t pitch, int y, int x0, const int (&c)[N]) {
  constexpr int SB = BITS == 8 ? 1 : 2;
  constexpr int VB = N * SB;
  char* at = static_cast<char*>(base) + y * pitch + (size_t)x0 * SB;
  if ((reinterpret_cast<uintptr_t>(at) & (VB - 1)) == 0) {
    constexpr int PER = 4 / SB;
    uint32_t wd[VB / 4];
#pragma unroll
    for (int i = 0; i < VB / 4; ++i) wd[i] = 0u;
#pragma unroll
    for (int k = 0; k < N; ++k) wd[k / PER] |= (uint32_t)c[k] << (8 * SB * (k % PER));
    if constexpr (VB == 4) *reinterpret_cast<uint32_t*>(at) = wd[0];
    else if constexpr (VB == 8) *reinterpret_cast<u32x2*>(at) = u32x2{wd[0], wd[1]};
    else *reinterpret_cast<u32x4*>(at) = u32x4{wd[0], wd[1], wd[2], wd[3]};
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) Code<BITS>::put(base, pitch, y, x0 + k, c[k]);
  }
}

// ---- unpack: four consecutive padded pixels of one row of each plane per thread ----
// (Y'CbCr -> R'G'B': Y' = (Y - yo) / ys, C' = (C - co) / cs with the range's scale and
//  offset, R = Y' + 2(1-Kr) Cr', B = Y' + 2(1-Kb) Cb', G = Y' - 2Kb(1-Kb)/Kg Cb' - 2Kr(1-Kr)/Kg Cr')
// 4:2:0 chroma is first blended between its two nearest chroma rows (3/4, 1/4), then
// along the row: left siting (CTR false) takes chroma column j at luma column 2j and the
// mean of columns j, j+1 at 2j+1; centre siting takes 3/4 of column j and 1/4 of column
// j-1 (at 2j) or j+1 (at 2j+1).  Edge columns and rows are replicated.
template <int BITS, bool C420, bool CTR>
__device__ __forceinline__ void unpack_px4(const Frame& f, const Inv& m, float* __restrict__ rgb, int hp,
                                           int wp, int y, int x0) {
  const int sy = min(y, f.h - 1);
  const int hc = C420 ? (f.h >> 1) : f.h;
  const int wc = C420 ? (f.w >> 1) : f.w;
  // vertical chroma neighbour of this luma row (4:2:0, chroma sited between rows 2i, 2i+1)
  const int ci = C420 ? (sy >> 1) : sy;
  const int ci2 = C420 ? ((sy & 1) ? min(ci + 1, hc - 1) : max(ci - 1, 0)) : ci;
  float r[4], g[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int sx = min(x0 + k, f.w - 1);
    const float yv = Code<BITS>::get(f.p[0], f.pitch[0], sy, sx);
    float cb, cr;
    if (C420) {
      const int cj = sx >> 1;
      const float cb0 = 0.75f * Code<BITS>::get(f.p[1], f.pitch[1], ci, cj) +
                        0.25f * Code<BITS>::get(f.p[1], f.pitch[1], ci2, cj);
      const float cr0 = 0.75f * Code<BITS>::get(f.p[2], f.pitch[2], ci, cj) +
                        0.25f * Code<BITS>::get(f.p[2], f.pitch[2], ci2, cj);
      if (CTR) {
        const int cn = (sx & 1) ? min(cj + 1, wc - 1) : max(cj - 1, 0);
        const float cbn = 0.75f * Code<BITS>::get(f.p[1], f.pitch[1], ci, cn) +
                          0.25f * Code<BITS>::get(f.p[1], f.pitch[1], ci2, cn);
        const float crn = 0.75f * Code<BITS>::get(f.p[2], f.pitch[2], ci, cn) +
                          0.25f * Code<BITS>::get(f.p[2], f.pitch[2], ci2, cn);
        cb = 0.75f * cb0 + 0.25f * cbn;
        cr = 0.75f * cr0 + 0.25f * crn;
      } else if (sx & 1) {
        const int cj1 = min(cj + 1, wc - 1);
        const float cb1 = 0.75f * Code<BITS>::get(f.p[1], f.pitch[1], ci, cj1) +
                          0.25f * Code<BITS>::get(f.p[1], f.pitch[1], ci2, cj1);
        const float cr1 = 0.75f * Code<BITS>::get(f.p[2], f.pitch[2], ci, cj1) +
                          0.25f * Code<BITS>::get(f.p[2], f.pitch[2], ci2, cj1);
        cb = 0.5f * (cb0 + cb1);
        cr = 0.5f * (cr0 + cr1);
      } else {
        cb = cb0;
        cr = cr0;
      }
    } else {
      cb = Code<BITS>::get(f.p[1], f.pitch[1], ci, sx);
      cr = Code<BITS>::get(f.p[2], f.pitch[2], ci, sx);
    }
    const float yn = (yv - m.yo) * m.ys;
    const float cbn = (cb - m.co) * m.cs;
    const float crn = (cr - m.co) * m.cs;
    r[k] = fmaf(m.rcr, crn, yn);
    b[k] = fmaf(m.bcb, cbn, yn);
    g[k] = fmaf(-m.gcr, crn, fmaf(-m.gcb, cbn, yn));
  }
  (void)wc;
  const size_t plane = (size_t)hp * wp;
  float* o = rgb + (size_t)y * wp + x0;
  st4(o, f32x4{r[0], r[1], r[2], r[3]});
  st4(o + plane, f32x4{g[0], g[1], g[2], g[3]});
  st4(o + 2 * plane, f32x4{b[0], b[1], b[2], b[3]});
}

// Two codes of row y from column x0 (x0 even, x0 + 1 < w): one load when aligned.
template <int BITS>
__device__ __forceinline__ void code_pair(const void* base, int64_t pitch, int y, int x0, float (&v)[2]) {
  constexpr uint32_t mask = BITS == 8 ? 0xFFu : 0x3FFu;
  const char* at = static_cast<const char*>(base) + y * pitch + (size_t)x0 * (BITS == 8 ? 1 : 2);
  if ((reinterpret_cast<uintptr_t>(at) & (BITS == 8 ? 1 : 3)) == 0) {
    const uint32_t wd = BITS == 8 ? (uint32_t)*reinterpret_cast<const uint16_t*>(at)
                                  : *reinterpret_cast<const uint32_t*>(at);
    v[0] = (float)(wd & mask);
    v[1] = (float)((wd >> (BITS == 8 ? 8 : 16)) & mask);
  } else {
    v[0] = Code<BITS>::get(base, pitch, y, x0);
    v[1] = Code<BITS>::get(base, pitch, y, x0 + 1);
  }
}

// Four consecutive padded pixels of row y per thread, so that each of the wave's
// float4 stores covers one contiguous kilobyte of an output plane.  Runs fully inside
// the frame read each plane row with vector loads (luma 4 codes; 4:2:0 chroma the 2 + 1
// codes the bilinear filter needs from rows ci and ci2); runs that reach into the
// padding use the per-pixel form.
template <int BITS, bool C420, bool CTR = false>
__device__ __forceinline__ void unpack4(const Frame& f, const Inv& m, float* __restrict__ rgb, int hp, int wp,
                                        int gid) {
  const int groups_per_row = wp >> 2;   // wp is a multiple of 4
  if (gid >= groups_per_row * hp) return;
  const int y = gid / groups_per_row;
  const int x0 = (gid - y * groups_per_row) << 2;
  if (x0 + 4 > f.w) {
    unpack_px4<BITS, C420, CTR>(f, m, rgb, hp, wp, y, x0);
    return;
  }
  const int sy = min(y, f.h - 1);
  float yv[4], cb[4], cr[4];
  code_run<BITS, 4>(f.p[0], f.pitch[0], sy, x0, f.w, yv);
  if (C420) {
    const int hc = f.h >> 1, wc = f.w >> 1;
    const int ci = sy >> 1;
    const int ci2 = (sy & 1) ? min(ci + 1, hc - 1) : max(ci - 1, 0);
    const int c0 = x0 >> 1, c2 = min(c0 + 2, wc - 1), cl = max(c0 - 1, 0);
#pragma unroll
    for (int pl = 1; pl <= 2; ++pl) {
      // vb[i]: chroma column c0 + i - 1 (cl, c0, c0 + 1, c2) blended between rows ci, ci2
      float top[2], bot[2], vb[4];
      code_pair<BITS>(f.p[pl], f.pitch[pl], ci, c0, top);
      code_pair<BITS>(f.p[pl], f.pitch[pl], ci2, c0, bot);
#pragma unroll
      for (int i = 0; i < 2; ++i) vb[1 + i] = 0.75f * top[i] + 0.25f * bot[i];
      vb[3] = 0.75f * Code<BITS>::get(f.p[pl], f.pitch[pl], ci, c2) +
              0.25f * Code<BITS>::get(f.p[pl], f.pitch[pl], ci2, c2);
      float* c = pl == 1 ? cb : cr;
      if (CTR) {
        vb[0] = 0.75f * Code<BITS>::get(f.p[pl], f.pitch[pl], ci, cl) +
                0.25f * Code<BITS>::get(f.p[pl], f.pitch[pl], ci2, cl);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int j = 1 + (k >> 1);                  // this pixel's chroma column
          c[k] = 0.75f * vb[j] + 0.25f * vb[(k & 1) ? j + 1 : j - 1];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = (k & 1) ? 0.5f * (vb[1 + (k >> 1)] + vb[2 + (k >> 1)]) : vb[1 + (k >> 1)];
      }
    }
  } else {
    code_run<BITS, 4>(f.p[1], f.pitch[1], sy, x0, f.w, cb);
    code_run<BITS, 4>(f.p[2], f.pitch[2], sy, x0, f.w, cr);
  }
  float r[4], g[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float yn = (yv[k] - m.yo) * m.ys;
    const float cbn = (cb[k] - m.co) * m.cs;
    const float crn = (cr[k] - m.co) * m.cs;
    r[k] = fmaf(m.rcr, crn, yn);
    b[k] = fmaf(m.bcb, cbn, yn);
    g[k] = fmaf(-m.gcr, crn, fmaf(-m.gcb, cbn, yn));
  }
  const size_t plane = (size_t)hp * wp;
  float* o = rgb + (size_t)y * wp + x0;
  st4(o, f32x4{r[0], r[1], r[2], r[3]});
  st4(o + plane, f32x4{g[0], g[1], g[2], g[3]});
  st4(o + 2 * plane, f32x4{b[0], b[1], b[2], b[3]});
}

__device__ __forceinline__ void unpack_any(const Frame& f, const Inv& m, float* rgb, int hp, int wp, int gid) {
  if (f.bits == 8) {
    if (f.chroma != 420) unpack4<8, false>(f, m, rgb, hp, wp, gid);
    else if (f.centre) unpack4<8, true, true>(f, m, rgb, hp, wp, gid);
    else unpack4<8, true>(f, m, rgb, hp, wp, gid);
  } else {
    if (f.chroma != 420) unpack4<10, false>(f, m, rgb, hp, wp, gid);
    else if (f.centre) unpack4<10, true, true>(f, m, rgb, hp, wp, gid);
    else unpack4<10, true>(f, m, rgb, hp, wp, gid);
  }
}

template <int BITS, bool C420, bool CTR>
__global__ __launch_bounds__(256) void k_unpack(Frame f, Inv m, float* __restrict__ rgb, int hp,
                                                int wp) {
  unpack4<BITS, C420, CTR>(f, m, rgb, hp, wp, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_unpack_batch(const UnpackJob* __restrict__ jobs,
                                                      const int* __restrict__ count) {
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const UnpackJob& J = jobs[find_job(jobs, njobs, item)];
    unpack_any(J.f, J.m, J.rgb, J.hp, J.wp, (item - J.item_begin) * 256 + threadIdx.x);
  }
}

// ---- pack ----
__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

__device__ __forceinline__ int quant(float v, float maxc) {
  return (int)fminf(fmaxf(floorf(v + 0.5f), 0.0f), maxc);
}

// 4:2:0: one thread per chroma sample, i.e. one 2x2 luma block and the chroma filter:
// left siting (1/4, 1/2, 1/4) over columns 2j-1..2j+1 times (1/2, 1/2) over rows 2i,
// 2i+1; centre siting (CTR) the mean of the 2x2 block.
template <int BITS, bool CTR>
__device__ __forceinline__ void pack420_px(const FrameOut& f, const Fwd& m,
                                           const float* __restrict__ rgb, int rh, int rw, int gid) {
  const int wc = f.w >> 1, hc = f.h >> 1;
  if (gid >= wc * hc) return;
  const int i = gid / wc, j = gid - i * wc;
  const size_t plane = (size_t)rh * rw;
  float cbs = 0.0f, crs = 0.0f;
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    const int yy = 2 * i + dy;
    const float* row = rgb + (size_t)yy * rw;
#pragma unroll
    for (int dx = CTR ? 0 : -1; dx <= 1; ++dx) {
      const int xx = max(2 * j + dx, 0);
      const float R = clamp01(row[xx]);
      const float G = clamp01(row[xx + plane]);
      const float B = clamp01(row[xx + 2 * plane]);
      const float Yn = fmaf(m.kb, B, fmaf(m.kg, G, m.kr * R));
      const float wgt = CTR || dx == 0 ? 0.25f : 0.125f;
      cbs = fmaf(wgt, (B - Yn) * m.cbs, cbs);
      crs = fmaf(wgt, (R - Yn) * m.crs, crs);
      if (dx >= 0) Code<BITS>::put(f.p[0], f.pitch[0], yy, xx, quant(fmaf(Yn, m.ys, m.yo), m.maxc));
    }
  }
  Code<BITS>::put(f.p[1], f.pitch[1], i, j, quant(fmaf(cbs, m.cs, m.co), m.maxc));
  Code<BITS>::put(f.p[2], f.pitch[2], i, j, quant(fmaf(crs, m.cs, m.co), m.maxc));
}

template <int BITS>
__device__ __forceinline__ void pack444_px(const FrameOut& f, const Fwd& m,
                                           const float* __restrict__ rgb, int rh, int rw, int gid) {
  if (gid >= f.w * f.h) return;
  const int y = gid / f.w, x = gid - y * f.w;
  const size_t plane = (size_t)rh * rw;
  const float* px = rgb + (size_t)y * rw + x;
  const float R = clamp01(px[0]), G = clamp01(px[plane]), B = clamp01(px[2 * plane]);
  const float Yn = fmaf(m.kb, B, fmaf(m.kg, G, m.kr * R));
  Code<BITS>::put(f.p[0], f.pitch[0], y, x, quant(fmaf(Yn, m.ys, m.yo), m.maxc));
  Code<BITS>::put(f.p[1], f.pitch[1], y, x, quant(fmaf((B - Yn) * m.cbs, m.cs, m.co), m.maxc));
  Code<BITS>::put(f.p[2], f.pitch[2], y, x, quant(fmaf((R - Yn) * m.crs, m.cs, m.co), m.maxc));
}

// Four chroma samples of chroma row i per thread (a 2 x 8 luma block): each R'G'B' row
// is read as two float4 vectors plus the left neighbour, the codes are written as
// vector runs.  Blocks that reach past the frame width use the per-sample form.
template <int BITS, bool CTR = false>
__device__ __forceinline__ void pack420_x4(const FrameOut& f, const Fwd& m, const float* __restrict__ rgb,
                                           int rh, int rw, int gid) {
  const int wc = f.w >> 1, hc = f.h >> 1;
  const int gpr = (wc + 3) >> 2;
  if (gid >= gpr * hc) return;
  const int i = gid / gpr, j0 = (gid - i * gpr) << 2;
  if (j0 + 4 > wc) {
    for (int j = j0; j < wc; ++j) pack420_px<BITS, CTR>(f, m, rgb, rh, rw, i * wc + j);
    return;
  }
  const size_t plane = (size_t)rh * rw;
  const int x0 = 2 * j0;
  float cbs[4] = {0.0f, 0.0f, 0.0f, 0.0f}, crs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    const int yy = 2 * i + dy;
    const float* row = rgb + (size_t)yy * rw;
    float R[9], G[9], B[9];           // columns x0 - 1 .. x0 + 7
    const int xl = max(x0 - 1, 0);
    R[0] = row[xl];
    G[0] = row[xl + plane];
    B[0] = row[xl + 2 * plane];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x4 r4 = ld4(row + x0 + 4 * h), g4 = ld4(row + plane + x0 + 4 * h),
                  b4 = ld4(row + 2 * plane + x0 + 4 * h);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        R[1 + 4 * h + k] = r4[k];
        G[1 + 4 * h + k] = g4[k];
        B[1 + 4 * h + k] = b4[k];
      }
    }
    float Yn[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      R[c] = clamp01(R[c]);
      G[c] = clamp01(G[c]);
      B[c] = clamp01(B[c]);
      Yn[c] = fmaf(m.kb, B[c], fmaf(m.kg, G[c], m.kr * R[c]));
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int dx = CTR ? 0 : -1; dx <= 1; ++dx) {
        const int c = 1 + 2 * jj + dx;
        const float wgt = CTR || dx == 0 ? 0.25f : 0.125f;
        cbs[jj] = fmaf(wgt, (B[c] - Yn[c]) * m.cbs, cbs[jj]);
        crs[jj] = fmaf(wgt, (R[c] - Yn[c]) * m.crs, crs[jj]);
      }
    int yc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) yc[k] = quant(fmaf(Yn[1 + k], m.ys, m.yo), m.maxc);
    code_store<BITS, 8>(f.p[0], f.pitch[0], yy, x0, yc);
  }
  int cbc[4], crc[4];
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    cbc[jj] = quant(fmaf(cbs[jj], m.cs, m.co), m.maxc);
    crc[jj] = quant(fmaf(crs[jj], m.cs, m.co), m.maxc);
  }
  code_store<BITS, 4>(f.p[1], f.pitch[1], i, j0, cbc);
  code_store<BITS, 4>(f.p[2], f.pitch[2], i, j0, crc);
}

// Eight consecutive pixels of row y per thread.
template <int BITS>
__device__ __forceinline__ void pack444_x8(const FrameOut& f, const Fwd& m, const float* __restrict__ rgb,
                                           int rh, int rw, int gid) {
  const int gpr = (f.w + 7) >> 3;
  if (gid >= gpr * f.h) return;
  const int y = gid / gpr, x0 = (gid - y * gpr) << 3;
  if (x0 + 8 > f.w) {
    for (int x = x0; x < f.w; ++x) pack444_px<BITS>(f, m, rgb, rh, rw, y * f.w + x);
    return;
  }
  const size_t plane = (size_t)rh * rw;
  const float* row = rgb + (size_t)y * rw + x0;
  int yc[8], cbc[8], crc[8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x4 r4 = ld4(row + 4 * h), g4 = ld4(row + plane + 4 * h), b4 = ld4(row + 2 * plane + 4 * h);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float R = clamp01(r4[k]), G = clamp01(g4[k]), B = clamp01(b4[k]);
      const float Yn = fmaf(m.kb, B, fmaf(m.kg, G, m.kr * R));
      yc[4 * h + k] = quant(fmaf(Yn, m.ys, m.yo), m.maxc);
      cbc[4 * h + k] = quant(fmaf((B - Yn) * m.cbs, m.cs, m.co), m.maxc);
      crc[4 * h + k] = quant(fmaf((R - Yn) * m.crs, m.cs, m.co), m.maxc);
    }
  }
  code_store<BITS, 8>(f.p[0], f.pitch[0], y, x0, yc);
  code_store<BITS, 8>(f.p[1], f.pitch[1], y, x0, cbc);
  code_store<BITS, 8>(f.p[2], f.pitch[2], y, x0, crc);
}

__device__ __forceinline__ void pack_any(const FrameOut& f, const Fwd& m, const float* rgb, int rh,
                                         int rw, int gid) {
  if (f.chroma == 420) {
    if (f.bits == 8) {
      if (f.centre) pack420_x4<8, true>(f, m, rgb, rh, rw, gid);
      else pack420_x4<8>(f, m, rgb, rh, rw, gid);
    } else {
      if (f.centre) pack420_x4<10, true>(f, m, rgb, rh, rw, gid);
      else pack420_x4<10>(f, m, rgb, rh, rw, gid);
    }
  } else {
    if (f.bits == 8) pack444_x8<8>(f, m, rgb, rh, rw, gid);
    else pack444_x8<10>(f, m, rgb, rh, rw, gid);
  }
}

template <int BITS, bool CTR>
__global__ __launch_bounds__(256) void k_pack420(FrameOut f, Fwd m, const float* __restrict__ rgb,
                                                 int rh, int rw) {
  pack420_x4<BITS, CTR>(f, m, rgb, rh, rw, blockIdx.x * 256 + threadIdx.x);
}

template <int BITS>
__global__ __launch_bounds__(256) void k_pack444(FrameOut f, Fwd m, const float* __restrict__ rgb,
                                                 int rh, int rw) {
  pack444_x8<BITS>(f, m, rgb, rh, rw, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_pack_batch(const PackJob* __restrict__ jobs,
                                                    const int* __restrict__ count) {
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const PackJob& J = jobs[find_job(jobs, njobs, item)];
    pack_any(J.f, J.m, J.rgb, J.rh, J.rw, (item - J.item_begin) * 256 + threadIdx.x);
  }
}

// ---- scene metric ----
// A thread takes runs of 16 adjacent luma codes of one row (one or two 16-byte loads
// where the row allows): it adds |Y_t - Y_{t-1}| into a register sum and bins the run
// into the workgroup's LDS histogram, one LDS atomic per stretch of equal bins
// (neighbouring codes of natural images mostly share a bin).  Workgroups then add their
// partial sums into the frame's accumulators with one global atomic per used bin.

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int kRun = 16;   // luma codes per thread and step

// Codes x0 .. x0+15 of row y (zero past the row end w).
template <int BITS>
__device__ __forceinline__ void luma_run(const void* base, int64_t pitch, int y, int x0, int w,
                                         uint32_t (&c)[kRun]) {
  constexpr int SB = BITS == 8 ? 1 : 2;
  constexpr uint32_t mask = BITS == 8 ? 0xFFu : 0x3FFu;
  const char* at = static_cast<const char*>(base) + y * pitch + (size_t)x0 * SB;
  if (x0 + kRun <= w && (reinterpret_cast<uintptr_t>(at) & 15) == 0) {
    uint32_t wd[kRun * SB / 4];
#pragma unroll
    for (int v = 0; v < SB; ++v) {
      const u32x4 t = reinterpret_cast<const u32x4*>(at)[v];
#pragma unroll
      for (int i = 0; i < 4; ++i) wd[4 * v + i] = t[i];
    }
#pragma unroll
    for (int k = 0; k < kRun; ++k) {
      constexpr int PER = 4 / SB;
      c[k] = (wd[k / PER] >> (8 * SB * (k % PER))) & mask;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kRun; ++k) c[k] = x0 + k < w ? (uint32_t)Code<BITS>::get(base, pitch, y, x0 + k) : 0u;
  }
}

// Codes x0 .. x0+n-1 (n = min(16, w - x0)) written to row y of a luma copy.
template <int BITS>
__device__ __forceinline__ void luma_run_store(void* base, int64_t pitch, int y, int x0, int w,
                                               const uint32_t (&c)[kRun]) {
  constexpr int SB = BITS == 8 ? 1 : 2;
  char* at = static_cast<char*>(base) + y * pitch + (size_t)x0 * SB;
  if (x0 + kRun <= w && (reinterpret_cast<uintptr_t>(at) & 15) == 0) {
    constexpr int PER = 4 / SB;
    uint32_t wd[kRun / PER];
#pragma unroll
    for (int i = 0; i < kRun / PER; ++i) wd[i] = 0u;
#pragma unroll
    for (int k = 0; k < kRun; ++k) wd[k / PER] |= c[k] << (8 * SB * (k % PER));
#pragma unroll
    for (int v = 0; v < SB; ++v)
      reinterpret_cast<u32x4*>(at)[v] = u32x4{wd[4 * v], wd[4 * v + 1], wd[4 * v + 2], wd[4 * v + 3]};
  } else {
#pragma unroll
    for (int k = 0; k < kRun; ++k)
      if (x0 + k < w) Code<BITS>::put(base, pitch, y, x0 + k, (int)c[k]);
  }
}

// One run: SAD against the previous luma into *s, histogram into lh, optional copy.
template <int BITS>
__device__ __forceinline__ void scene_run(const Frame& cur, const void* prev_y, int64_t prev_pitch,
                                          void* luma_save, int64_t save_pitch, int y, int x0,
                                          uint32_t* lh, uint32_t& s) {
  constexpr int SH = BITS - 6;
  uint32_t c[kRun];
  luma_run<BITS>(cur.p[0], cur.pitch[0], y, x0, cur.w, c);
  if (prev_y != nullptr) {
    uint32_t p[kRun];
    luma_run<BITS>(prev_y, prev_pitch, y, x0, cur.w, p);
#pragma unroll
    for (int k = 0; k < kRun; ++k) s += (uint32_t)abs((int)c[k] - (int)p[k]);   // zero past the row end
  }
  const int n = min(kRun, cur.w - x0);
  uint32_t bin = c[0] >> SH, cnt = 1u;
#pragma unroll
  for (int k = 1; k < kRun; ++k) {
    if (k < n) {
      const uint32_t bk = c[k] >> SH;
      if (bk == bin) {
        ++cnt;
      } else {
        atomicAdd(&lh[bin], cnt);
        bin = bk;
        cnt = 1u;
      }
    }
  }
  atomicAdd(&lh[bin], cnt);
  if (luma_save != nullptr) luma_run_store<BITS>(luma_save, save_pitch, y, x0, cur.w, c);
}

// Runs [r0, r1) of a frame whose rows hold nrun runs each, strided over the workgroup.
template <int BITS>
__device__ __forceinline__ uint32_t scene_runs(const SceneJob& J, int nrun, int r0, int r1, int stride,
                                               uint32_t* lh) {
  uint32_t s = 0u;
  for (int r = r0 + (int)threadIdx.x; r < r1; r += stride) {
    const int y = r / nrun, x0 = (r - y * nrun) * kRun;
    scene_run<BITS>(J.cur, J.prev_y, J.prev_pitch, J.luma_save, J.luma_save_pitch, y, x0, lh, s);
  }
  return s;
}

// Adds the workgroup's partial SAD and histogram to the frame's accumulators.
__device__ __forceinline__ void scene_flush(uint32_t s, bool has_prev, uint32_t* lh, uint32_t* lsad,
                                            uint64_t* sad, uint32_t* hist) {
  if (has_prev) {
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lsad[threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 64 && lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
  if (has_prev && threadIdx.x == 0) {
    const uint64_t tot = (uint64_t)lsad[0] + lsad[1] + lsad[2] + lsad[3];
    if (tot) atomicAdd(reinterpret_cast<unsigned long long*>(sad), (unsigned long long)tot);
  }
}

// Frame t starts a scene when SAD > T * 2^(bits-8) * N and HD * den > 2 N num.  Run by
// one wave of 64 lanes (lane = histogram bin) after the accumulating launch.
__device__ __forceinline__ void scene_decide(const SceneJob& J, bool has_prev) {
  const int t = threadIdx.x;
  const uint64_t n_pix = (uint64_t)J.cur.w * (uint64_t)J.cur.h;
  const uint32_t h = J.hist[t];
  uint32_t d = 0;
  if (has_prev) d = (uint32_t)abs((int)h - (int)J.hist_prev[t]);
  d = wave_sum(d);
  if (J.hist_save != nullptr) J.hist_save[t] = h;
  if (t == 0) {
    const uint64_t sad = *J.sad;
    uint32_t c;
    if (!has_prev) {
      c = 1u;
      d = 0u;
    } else {
      const uint64_t thr = (uint64_t)J.rule.mad_thresh_8bit * (uint64_t)(1u << (J.cur.bits - 8)) * n_pix;
      const bool mad_ok = sad > thr;
      const bool hist_ok = (uint64_t)d * (uint64_t)J.rule.hist_den > 2ull * n_pix * (uint64_t)J.rule.hist_num;
      c = (J.rule.enable && mad_ok && hist_ok) ? 1u : 0u;
    }
    if (J.external > 0) c = 1u;
    if (J.sad_save != nullptr) *J.sad_save = sad;
    *J.hd = d;
    *J.cut = c;
  }
}

__global__ void k_scene_clear(uint64_t* sad, uint32_t* hist) {
  const int t = threadIdx.x;
  if (t < 64) hist[t] = 0u;
  if (t == 0) *sad = 0ull;
}

// One frame: the workgroups split the frame's runs into contiguous shares and add into
// the accumulators.  (A grid-wide "last workgroup decides" tail would need a device
// fence per workgroup, which writes back the L2 and costs more than a second launch.)
template <int BITS, bool HAS_PREV>
__global__ __launch_bounds__(256) void k_scene(SceneJob J) {
  __shared__ uint32_t lh[64];
  __shared__ uint32_t lsad[4];
  if (threadIdx.x < 64) lh[threadIdx.x] = 0u;
  __syncthreads();
  const int nrun = (J.cur.w + kRun - 1) / kRun, total = nrun * J.cur.h;
  const int per = (total + gridDim.x - 1) / gridDim.x;
  const int r0 = min(total, (int)blockIdx.x * per), r1 = min(total, r0 + per);
  uint32_t s = 0u;
  for (int b = r0; b < r1; b += 256) s += scene_runs<BITS>(J, nrun, b, min(r1, b + 256), 256, lh);
  scene_flush(s, HAS_PREV, lh, lsad, J.sad, J.hist);
}

// The decision, then (J.reset) the accumulators back to zero for the next frame.
__global__ void k_scene_final(SceneJob J, int has_prev) {
  scene_decide(J, has_prev != 0);
  if (J.reset) {
    J.hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *J.sad = 0ull;
  }
}

// Batched scene metric: clear every job's accumulators, accumulate row chunks, decide.
// (A frame's decision may read the previous frame's histogram from the same batch, so
// the decisions wait for the whole accumulate launch.)
__global__ __launch_bounds__(64) void k_scene_clear_batch(const SceneJob* __restrict__ jobs,
                                                          const int* __restrict__ count) {
  for (int j = blockIdx.x; j < count[0]; j += gridDim.x) {
    jobs[j].hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *jobs[j].sad = 0ull;
  }
}

__global__ __launch_bounds__(256) void k_scene_accum_batch(const SceneJob* __restrict__ jobs,
                                                           const int* __restrict__ count) {
  __shared__ uint32_t lh[64];
  __shared__ uint32_t lsad[4];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const SceneJob& J = jobs[find_job(jobs, njobs, item)];
    const int nrun = (J.cur.w + kRun - 1) / kRun;
    const int y0 = (item - J.item_begin) * kSceneRowsPerItem;
    const int r0 = y0 * nrun, r1 = min(y0 + kSceneRowsPerItem, J.cur.h) * nrun;
    if (threadIdx.x < 64) lh[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t s = J.cur.bits == 8 ? scene_runs<8>(J, nrun, r0, r1, 256, lh)
                                       : scene_runs<10>(J, nrun, r0, r1, 256, lh);
    scene_flush(s, J.prev_y != nullptr, lh, lsad, J.sad, J.hist);
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void k_scene_final_batch(const SceneJob* __restrict__ jobs,
                                                          const int* __restrict__ count) {
  for (int j = blockIdx.x; j < count[0]; j += gridDim.x) {
    const SceneJob& J = jobs[j];
    scene_decide(J, J.prev_y != nullptr && J.hist_prev != nullptr);
  }
}

}  // namespace

hipError_t launch_unpack(const Frame& f, float* rgb, int hp, int wp, hipStream_t s) {
  const Inv m = make_inv(f.bits, f.matrix, f.full);
  const int n = (wp >> 2) * hp;
  const dim3 grid((n + 255) / 256), blk(256);
  const bool c420 = f.chroma == 420, ctr = c420 && f.centre;
  if (f.bits == 8) {
    if (ctr) hipLaunchKernelGGL((k_unpack<8, true, true>), grid, blk, 0, s, f, m, rgb, hp, wp);
    else if (c420) hipLaunchKernelGGL((k_unpack<8, true, false>), grid, blk, 0, s, f, m, rgb, hp, wp);
    else hipLaunchKernelGGL((k_unpack<8, false, false>), grid, blk, 0, s, f, m, rgb, hp, wp);
  } else {
    if (ctr) hipLaunchKernelGGL((k_unpack<10, true, true>), grid, blk, 0, s, f, m, rgb, hp, wp);
    else if (c420) hipLaunchKernelGGL((k_unpack<10, true, false>), grid, blk, 0, s, f, m, rgb, hp, wp);
    else hipLaunchKernelGGL((k_unpack<10, false, false>), grid, blk, 0, s, f, m, rgb, hp, wp);
  }
  return hipGetLastError();
}

hipError_t launch_pack(const FrameOut& f, const float* rgb, int rh, int rw, hipStream_t s) {
  const Fwd m = make_fwd(f.bits, f.matrix, f.full);
  if (f.chroma == 420) {
    const int n = (((f.w >> 1) + 3) >> 2) * (f.h >> 1);
    const dim3 grid((n + 255) / 256), blk(256);
    if (f.bits == 8) {
      if (f.centre) hipLaunchKernelGGL((k_pack420<8, true>), grid, blk, 0, s, f, m, rgb, rh, rw);
      else hipLaunchKernelGGL((k_pack420<8, false>), grid, blk, 0, s, f, m, rgb, rh, rw);
    } else {
      if (f.centre) hipLaunchKernelGGL((k_pack420<10, true>), grid, blk, 0, s, f, m, rgb, rh, rw);
      else hipLaunchKernelGGL((k_pack420<10, false>), grid, blk, 0, s, f, m, rgb, rh, rw);
    }
  } else {
    const int n = ((f.w + 7) >> 3) * f.h;
    const dim3 grid((n + 255) / 256), blk(256);
    if (f.bits == 8) hipLaunchKernelGGL((k_pack444<8>), grid, blk, 0, s, f, m, rgb, rh, rw);
    else hipLaunchKernelGGL((k_pack444<10>), grid, blk, 0, s, f, m, rgb, rh, rw);
  }
  return hipGetLastError();
}

hipError_t launch_scene(const SceneJob& job, bool clear, hipStream_t s) {
  if (clear) hipLaunchKernelGGL(k_scene_clear, dim3(1), dim3(64), 0, s, job.sad, job.hist);
  const bool has_prev = job.prev_y != nullptr && job.hist_prev != nullptr;
  const int64_t runs = (int64_t)((job.cur.w + kRun - 1) / kRun) * job.cur.h;
  // about four runs per thread, at most 1024 workgroups
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (runs + 1023) / 1024));
  SceneJob J = job;
  if (!has_prev) J.prev_y = nullptr;
  if (job.cur.bits == 8) {
    if (has_prev) hipLaunchKernelGGL((k_scene<8, true>), dim3(blocks), dim3(256), 0, s, J);
    else hipLaunchKernelGGL((k_scene<8, false>), dim3(blocks), dim3(256), 0, s, J);
  } else {
    if (has_prev) hipLaunchKernelGGL((k_scene<10, true>), dim3(blocks), dim3(256), 0, s, J);
    else hipLaunchKernelGGL((k_scene<10, false>), dim3(blocks), dim3(256), 0, s, J);
  }
  hipLaunchKernelGGL(k_scene_final, dim3(1), dim3(64), 0, s, J, has_prev ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_unpack_batch(const UnpackJob* jobs, const int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_batch, dim3(kBatchGrid), dim3(256), 0, s, jobs, count);
  return hipGetLastError();
}

hipError_t launch_pack_batch(const PackJob* jobs, const int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_batch, dim3(kBatchGrid), dim3(256), 0, s, jobs, count);
  return hipGetLastError();
}

hipError_t launch_scene_batch(const SceneJob* jobs, const int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_scene_clear_batch, dim3(256), dim3(64), 0, s, jobs, count);
  hipLaunchKernelGGL(k_scene_accum_batch, dim3(kBatchGrid), dim3(256), 0, s, jobs, count);
  hipLaunchKernelGGL(k_scene_final_batch, dim3(256), dim3(64), 0, s, jobs, count);
  return hipGetLastError();
}

}  // namespace nv

// Network kernels (gfx950): 3x3 convolutions as implicit GEMM on MFMA, the thin output
// conv as MFMA "tap responses", and the 3 -> C input conv on the vector ALUs (the
// deformable convolution is in k_dcn.hip).
//
// Activations are NHWC.  A workgroup owns a tile of TH x 16 output pixels (TH = 4 waves
// x PB rows) and OB blocks of 16 output channels.  In the MFMA the weights are the A
// operand (rows = output channels) and the activations the B operand (columns = the
// 16 pixels of one tile row), so each lane ends up holding four consecutive output
// channels of one pixel.  Storage type (TIN / TOUT) and MFMA type (TC) are template
// parameters: float end to end, or float16 / bfloat16 storage and MFMA with float
// accumulation; the offset head reads 16-bit features and computes in float.
#include <algorithm>
#include <type_traits>

#include "nv_internal.h"
#include "nv_mma.h"

namespace nv {
namespace {

// Offset-head forms of a conv (see conv_tile).
enum { SPLIT_NONE = 0, SPLIT_W = 1, SPLIT_WX = 2 };

// Arguments shared by every image of a conv launch.
struct ConvLayer {
  const u32x4* wfrag;
  const float* bias;
  const float* oscale;   // FP8: per A row weight scale x activation scale
  const float* ainv;     // FP8: 1 / activation scale (device scalar)
  int ldy;      // channel stride of dst / res
  int cout;     // real output channels (EPI_OFFSET stores only these)
  int sig_lo;   // EPI_OFFSET: sigmoid on channels >= sig_lo
  int obtot;    // total 16-channel output blocks of the layer
  int ccout;    // EPI_SHUFFLE: channels of the high-resolution map
  int sv, sh;   // EPI_SHUFFLE: sub-pixel rows and columns (sub-pixel s -> row s / sh, column s % sh)
};

template <typename TC, int CCH, int PB>
struct ConvSmem {
  static constexpr int TH = 4 * PB;
  static constexpr int LDP = CCH + 16 / (int)sizeof(TC);   // LDS pixel stride (16-byte pad)
  // the input tile, or (FP8 tiles, whose storage type is float16) the staged 16-bit
  // output tile if that is larger
  static constexpr int NIN = (TH + 2) * (kTW + 2) * LDP;
  static constexpr int NOUT = std::is_same<TC, f8>::value ? TH * kTW * (CCH + 8) * 2 : 0;
  static constexpr int N = NIN > NOUT ? NIN : NOUT;
};

// Epilogue of a wave's part of a conv tile (rows y0 .. y0 + PB, output blocks obase ..
// obase + OB): bias (and, for FP8, the per-row output scale), then the layer's
// activation / residual / offset-head / pixel-shuffle store.
template <typename TOUT, int OB, int PB, int EPI>
__device__ __forceinline__ void conv_store(const ConvLayer& L, const ConvImg& im, const f32x4 (&acc)[PB][OB],
                                           int y0, int tx0, int obase, const float* oscale) {
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, j = lane & 15;
  TOUT* dst = static_cast<TOUT*>(im.dst);
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int gy = y0 + pb, gx = tx0 + j;
    if (gy >= im.H || gx >= im.W) continue;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = (obase + ob) * 16 + 4 * q;
      f32x4 v = oscale ? acc[pb][ob] * ld4(oscale + row) : acc[pb][ob];
      v += ld4(L.bias + row);
      const size_t at = ((size_t)gy * im.W + gx) * L.ldy + row;
      if (EPI == EPI_LRELU) {
        store4f<TOUT>(dst + at, lrelu4(v));
      } else if (EPI == EPI_RES) {
        v += load4f<TOUT>(static_cast<const TOUT*>(im.res) + at);
        store4f<TOUT>(dst + at, v);
      } else if (EPI == EPI_OFFSET) {
        if (row + 4 <= L.cout && (L.sig_lo & 3) == 0) {
          // whole group of four channels: offsets, or mask logits through the sigmoid
          if (row >= L.sig_lo) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = sigmoidf(v[r]);
          }
          store4f<TOUT>(dst + at, v);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = row + r;
            if (o < L.cout) dst[at + r] = (TOUT)(o >= L.sig_lo ? sigmoidf(v[r]) : v[r]);
          }
        }
      } else {  // EPI_SHUFFLE: A row 16*g + t is channel 16*(g % NB) + t at sub-pixel g / NB
        const int obg = obase + ob, nb = L.ccout >> 4;
        const int sp = obg / nb, c = 16 * (obg - sp * nb) + 4 * q;
        const int Y = L.sv * gy + sp / L.sh, X = L.sh * gx + sp % L.sh;
        store4f<TOUT>(dst + ((size_t)Y * (L.sh * im.W) + X) * L.ccout + c, lrelu4(v));
      }
    }
  }
}


// FP8 tile of a 64-channel float16 map (residual-block and pixel-shuffle convs).  The
// input tile is staged in LDS as e4m3 of x / s_act.  One MFMA step covers 128
// reduction indices, two taps x 64 channels: lane quarter q takes tap 2 st + q / 2,
// channels 32 (q % 2) .. +32.  The fifth step pairs tap 8 with a zero-weight tap (its
// lanes read tap 8's samples again, which are finite).  The accumulator is rescaled
// by s_w[row] x s_act in the epilogue.
// Epilogue through LDS for a tile holding all 64 output channels: each wave writes
// bias-added, activated (or skip-added, in float as in conv_store) results into the
// LDS tile in the storage type, then the workgroup copies whole pixels out in 16-byte
// pieces.  The arithmetic and rounding are conv_store's, so the results are
// bit-identical.
// Four 16-bit elements held raw in two dwords -> four floats.
template <typename TC>
__device__ __forceinline__ f32x4 raw4f(u32x2 r) {
  if constexpr (std::is_same<TC, f16>::value) {
    const f16x4 v = __builtin_bit_cast(f16x4, r);
    return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  } else {
    const bf16x4 v = __builtin_bit_cast(bf16x4, r);
    return f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  }
}

template <typename TC, int OBW, int RW, int PB, int EPI, typename TL = TC, bool PRE = false>
__device__ __forceinline__ void conv_store_staged(const ConvLayer& L, const ConvImg& im, const f32x4 (&acc)[RW][OBW],
                                                  int ty0, int tx0, int wr, int wo, TC* tile,
                                                  const float* oscale = nullptr,
                                                  const u32x2 (*resr)[OBW] = nullptr) {
  constexpr int C = 64, OLDP = C + 16 / (int)sizeof(TC), TH = 4 * PB;
  static_assert(TH * kTW * OLDP * (int)sizeof(TC) <= ConvSmem<TL, C, PB>::N * (int)sizeof(TL),
                "the output tile fits in the workgroup's LDS tile");
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, j = lane & 15;
  __syncthreads();   // every wave is done reading the input tile
#pragma unroll
  for (int pb = 0; pb < RW; ++pb) {
    const int r = wr * RW + pb, gy = ty0 + r, gx = tx0 + j;
    const bool inside = gy < im.H && gx < im.W;
#pragma unroll
    for (int ob = 0; ob < OBW; ++ob) {
      const int row = (wo * OBW + ob) * 16 + 4 * q;
      f32x4 v = oscale ? acc[pb][ob] * ld4(oscale + row) : acc[pb][ob];
      v += ld4(L.bias + row);
      if (EPI == EPI_LRELU) {
        v = lrelu4(v);
      } else if constexpr (PRE) {
        v += raw4f<TC>(resr[pb][ob]);   // skip values loaded before the main loop
      } else if (inside) {
        v += load4f<TC>(static_cast<const TC*>(im.res) + ((size_t)gy * im.W + gx) * C + row);
      }
      store4f<TC>(&tile[(r * kTW + j) * OLDP + row], v);
    }
  }
  __syncthreads();
  TC* dst = static_cast<TC*>(im.dst);
  constexpr int E = 16 / (int)sizeof(TC), NPC = C / E;      // elements per piece, pieces per pixel
  constexpr int NCHK = TH * kTW * NPC;
#pragma unroll
  for (int idx = (int)threadIdx.x; idx < NCHK; idx += 256) {
    const int px = idx / NPC, ck = idx - px * NPC;
    const int gy = ty0 + px / kTW, gx = tx0 + px % kTW;
    if (gy < im.H && gx < im.W) stu4(dst + ((size_t)gy * im.W + gx) * C + E * ck, ldu4(&tile[px * OLDP + E * ck]));
  }
}

// Pixel-shuffle epilogue through LDS: the workgroup's row blocks obase .. obase + 7
// are sub-pixels sp0 = obase / 4 and sp0 + 1 with all 64 channels each (four blocks per
// sub-pixel); each pass writes one sub-pixel's LReLU-ed results into the LDS tile and
// copies whole high-resolution pixels out (sub-pixel s at row s / sh, column s % sh of
// the sv x sh block).  Same arithmetic as conv_store.
template <typename TC, int OBW, int RW, int PB>
__device__ __forceinline__ void conv_store_shuffle_staged(const ConvLayer& L, const ConvImg& im,
                                                          const f32x4 (&acc)[RW][OBW], int ty0, int tx0, int wr,
                                                          int wo, int obase, TC* tile) {
  constexpr int C = 64, OLDP = C + 16 / (int)sizeof(TC), TH = 4 * PB;
  static_assert(TH * kTW * OLDP <= ConvSmem<TC, C, PB>::N, "a sub-pixel's tile fits in the input tile's LDS");
  constexpr int E = 16 / (int)sizeof(TC), NPC = C / E;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, j = lane & 15;
  const int sp0 = obase >> 2;
  TC* dst = static_cast<TC*>(im.dst);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    __syncthreads();   // the input tile, or the previous sub-pixel, is fully read
#pragma unroll
    for (int pb = 0; pb < RW; ++pb) {
      const int r = wr * RW + pb;
#pragma unroll
      for (int ob = 0; ob < OBW; ++ob) {
        const int g = obase + wo * OBW + ob;
        if ((g >> 2) - sp0 != s) continue;
        const int row = g * 16 + 4 * q;
        f32x4 v = acc[pb][ob];
        v += ld4(L.bias + row);
        store4f<TC>(&tile[(r * kTW + j) * OLDP + 16 * (g & 3) + 4 * q], lrelu4(v));
      }
    }
    __syncthreads();
    const int sp = sp0 + s;
#pragma unroll
    for (int idx = (int)threadIdx.x; idx < TH * kTW * NPC; idx += 256) {
      const int px = idx / NPC, ck = idx - px * NPC;
      const int gy = ty0 + px / kTW, gx = tx0 + px % kTW;
      if (gy < im.H && gx < im.W) {
        const int Y = L.sv * gy + sp / L.sh, X = L.sh * gx + sp % L.sh;
        stu4(dst + ((size_t)Y * (L.sh * im.W) + X) * C + E * ck, ldu4(&tile[px * OLDP + E * ck]));
      }
    }
  }
}

template <int OB, int PB, int EPI, int WO>
__device__ __forceinline__ void conv_tile_f8(const ConvLayer& L, const ConvImg& im, int ty0, int tx0, int obase,
                                             f8* tile) {
  constexpr int C = 64;
  constexpr int LDP = ConvSmem<f8, C, PB>::LDP;   // bytes per staged pixel
  constexpr int NST = 5;
  constexpr int RW = PB * WO, OBW = OB / WO;     // this wave's rows and output blocks
  static_assert(OB % WO == 0, "output blocks split evenly over the waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int wo = wave % WO, wr = wave / WO;

  f32x4 acc[RW][OBW];
#pragma unroll
  for (int pb = 0; pb < RW; ++pb)
#pragma unroll
    for (int ob = 0; ob < OBW; ++ob) acc[pb][ob] = zero4();

  const f16* src = static_cast<const f16*>(im.src0);
  if (im.sel != nullptr && *im.sel != 0u && im.alt0 != nullptr) src = static_cast<const f16*>(im.alt0);
  const float ainv = *L.ainv;

  constexpr int V = C / 8;
  constexpr int NV = (4 * PB + 2) * (kTW + 2) * V;
  constexpr int SB = 8;                     // loads in flight per thread while staging
  for (int i0 = 0; i0 < NV; i0 += SB * 256) {
    Raw8<f16> rb[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      rb[u].zero();
      if (idx < NV) {
        const int pix = idx / V, v = idx - pix * V;
        const int ly = pix / (kTW + 2), lx = pix - ly * (kTW + 2);
        const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
        if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) rb[u].load(src + ((size_t)gy * im.W + gx) * C + 8 * v);
      }
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      if (idx < NV) {
        const int pix = idx / V, v = idx - pix * V;
        f32x4 lo, hi;
        rb[u].to_f32(lo, hi);
        *reinterpret_cast<u32x2*>(&tile[pix * LDP + 8 * v]) = u32x2{f8x4_pack(lo * ainv), f8x4_pack(hi * ainv)};
      }
    }
  }
  __syncthreads();

  // the step loop stays rolled: unrolled, the compiler hoists all five steps' 32-byte
  // weight fragments (160 registers) and occupancy drops to one or two waves per SIMD
  const f8* tbase = &tile[((wr * RW) * (kTW + 2) + j) * LDP + 32 * (q & 1)];
  auto tap_off = [&](int st) {
    const int tap = min(2 * st + (q >> 1), 8);
    const int dy = tap / 3, dx = tap - 3 * dy;
    return (dy * (kTW + 2) + dx) * LDP;
  };
  const u32x8* wbase = reinterpret_cast<const u32x8*>(L.wfrag) + (size_t)(obase + wo * OBW) * 64 + lane;
  u32x8 wa0[OBW], xb0[RW], wa1[OBW], xb1[RW];
  auto fetch = [&](int st, u32x8 (&wa)[OBW], u32x8 (&xb)[RW]) {
    const u32x8* wp = wbase + (size_t)st * L.obtot * 64;
#pragma unroll
    for (int ob = 0; ob < OBW; ++ob) wa[ob] = wp[ob * 64];
    const int o = tap_off(st);
#pragma unroll
    for (int pb = 0; pb < RW; ++pb) xb[pb] = ldu8(tbase + o + pb * (kTW + 2) * LDP);
  };
  auto mma = [&](const u32x8 (&wa)[OBW], const u32x8 (&xb)[RW]) {
#pragma unroll
    for (int pb = 0; pb < RW; ++pb)
#pragma unroll
      for (int ob = 0; ob < OBW; ++ob) acc[pb][ob] = Mma<f8>::step(wa[ob], xb[pb], acc[pb][ob]);
  };
  // two register buffers, step i+1 loading while step i multiplies
  fetch(0, wa0, xb0);
#pragma unroll 1
  for (int st = 0; st < NST; st += 2) {
    if (st + 1 < NST) fetch(st + 1, wa1, xb1);
    mma(wa0, xb0);
    if (st + 1 < NST) {
      if (st + 2 < NST) fetch(st + 2, wa0, xb0);
      mma(wa1, xb1);
    }
  }
  if constexpr (OB == 4 && (EPI == EPI_LRELU || EPI == EPI_RES)) {
    if (L.obtot == OB && L.ldy == 16 * OB) {   // all 64 channels: whole pixels through LDS
      conv_store_staged<f16, OBW, RW, PB, EPI, f8>(L, im, acc, ty0, tx0, wr, wo, reinterpret_cast<f16*>(tile),
                                                   L.oscale);
      return;
    }
  }
  conv_store<f16, OBW, RW, EPI>(L, im, acc, ty0 + wr * RW, tx0, obase + wo * OBW, L.oscale);
}

// One output tile: rows [ty0, ty0 + 4 PB), columns [tx0, tx0 + 16), output blocks
// [obase, obase + OB).  Called by all 256 threads; contains block-wide barriers.
//
// SPLIT selects the float-class offset head on float16 MFMA: the weights are carried
// as two float16 parts per fragment (hi = f16(s w), lo = f16(s w - hi), s a power of
// two), each A fragment position holding the pair, so every product of a float16
// input with w is formed from 22 weight bits, exactly, and accumulated in float; the
// epilogue multiplies by 1/s.  SPLIT_W: inputs are float16 (or bfloat16 converted
// exactly) maps.  SPLIT_WX: the single float input is staged as two chunks, its
// float16 part and the float16 of the remainder, against the same weights (the
// remainder against their hi part only).
//
// WO splits the workgroup's four waves over the output blocks: each wave takes OB / WO
// blocks and PB * WO rows, so per MFMA a wave fetches 1/(PB WO) weight fragments from
// L1/L2 and 1/(OB/WO) activation fragments from LDS (WO = 2 balances the two).
template <typename TIN, typename TC, typename TOUT, int CCH, int NCHUNK, int OB, int PB, int EPI, int SPLIT = 0,
          int WO = 1>
__device__ __forceinline__ void conv_tile(const ConvLayer& L, const ConvImg& im, int ty0, int tx0,
                                          int obase, TC* tile) {
  if constexpr (std::is_same<TC, f8>::value) {
    static_assert(std::is_same<TIN, f16>::value && std::is_same<TOUT, f16>::value && CCH == 64 && NCHUNK == 1,
                  "FP8 convs read and write 64-channel float16 maps");
    conv_tile_f8<OB, PB, EPI, WO>(L, im, ty0, tx0, obase, tile);
    return;
  } else {
  constexpr int KG = Mma<TC>::KG;           // channels per MFMA step group
  constexpr int QE = KG / 4;                // channels per lane quarter
  constexpr int LDP = ConvSmem<TC, CCH, PB>::LDP;
  constexpr int NCG = CCH / KG;
  constexpr int NKG = NCHUNK * NCG;
  constexpr int AS = SPLIT ? 2 : 1;         // A fragments per output block and step
  constexpr int RW = PB * WO, OBW = OB / WO;  // this wave's rows and output blocks
  static_assert(SPLIT == 0 || std::is_same<TC, f16>::value, "the split head runs on float16 MFMA");
  static_assert(SPLIT != SPLIT_WX || (NCHUNK == 2 && std::is_same<TIN, float>::value), "SPLIT_WX stages hi / lo");
  static_assert(OB % WO == 0, "output blocks split evenly over the waves");
  const int wobtot = L.obtot * AS;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int wo = wave % WO, wr = wave / WO;

  f32x4 acc[RW][OBW];
#pragma unroll
  for (int pb = 0; pb < RW; ++pb)
#pragma unroll
    for (int ob = 0; ob < OBW; ++ob) acc[pb][ob] = zero4();

  constexpr bool kStaged = std::is_same<TIN, TC>::value && std::is_same<TOUT, TC>::value && SPLIT == 0 &&
                           NCHUNK == 1 && CCH == 64 && OB == 4 && (EPI == EPI_LRELU || EPI == EPI_RES);
  const bool staged_rt = L.obtot == OB && L.ldy == 16 * OB;
  // 16-bit residual conv with the staged epilogue: the skip values of this lane's
  // outputs are requested before the main loop, so their HBM latency is hidden behind
  // it instead of following the last MFMA (same arithmetic; two registers per output
  // fragment)
  constexpr bool kPre = kStaged && EPI == EPI_RES && sizeof(TC) == 2;
  u32x2 resr[RW][kPre ? OBW : 1];
  if constexpr (kPre) {
#pragma unroll
    for (int pb = 0; pb < RW; ++pb) {
      const int gy = ty0 + wr * RW + pb, gx = tx0 + j;
      const bool inside = staged_rt && gy < im.H && gx < im.W;
#pragma unroll
      for (int ob = 0; ob < OBW; ++ob) {
        const int row = (wo * OBW + ob) * 16 + 4 * q;
        resr[pb][ob] = inside ? *reinterpret_cast<const u32x2*>(static_cast<const TC*>(im.res) +
                                                                 ((size_t)gy * im.W + gx) * 64 + row)
                              : u32x2{0u, 0u};
      }
    }
  }

  const TIN* src0 = static_cast<const TIN*>(im.src0);
  const TIN* src1 = static_cast<const TIN*>(im.src1);
  if (im.sel != nullptr && *im.sel != 0u) {
    if (im.alt0 != nullptr) src0 = static_cast<const TIN*>(im.alt0);
    if (im.alt1 != nullptr) src1 = static_cast<const TIN*>(im.alt1);
  }

#pragma unroll
  for (int ch = 0; ch < NCHUNK; ++ch) {
    const TIN* src = (ch == 0 || SPLIT == SPLIT_WX) ? src0 : src1;
    if (ch) __syncthreads();
    // staging: a thread loads up to SB vectors of 8 channels before storing any of
    // them, so its global loads are in flight together
    constexpr int V = CCH / 8;
    constexpr int NV = (4 * PB + 2) * (kTW + 2) * V;
    constexpr int SB = std::is_same<TIN, float>::value ? 2 : 8;
    for (int i0 = 0; i0 < NV; i0 += SB * 256) {
      Raw8<TIN> rb[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 256 + (int)threadIdx.x;
        rb[u].zero();
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          const int ly = pix / (kTW + 2), lx = pix - ly * (kTW + 2);
          const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
          if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) rb[u].load(src + ((size_t)gy * im.W + gx) * CCH + 8 * v);
        }
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 256 + (int)threadIdx.x;
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          TC* dstp = &tile[pix * LDP + 8 * v];
          if constexpr (SPLIT == SPLIT_WX) copy8_split(dstp, rb[u], ch);
          else raw8_store<TIN, TC>(dstp, rb[u]);
        }
      }
    }
    __syncthreads();

    // (tap, channel group) steps, software-pipelined: the fragments of later steps are
    // loading while the MFMAs of step i run (float: one step ahead; 16-bit: A two steps
    // and B one step ahead, see below).
    constexpr int NIT = 9 * NCG;
    const u32x4* wbase = L.wfrag + ((size_t)(ch * NCG) * wobtot + (obase + wo * OBW) * AS) * 64 + lane;
    const size_t wstride_tap = (size_t)NKG * wobtot * 64;
    const TC* tbase = &tile[((wr * RW) * (kTW + 2) + j) * LDP + QE * q];
    u32x4 wa0[OBW * AS], xb0[RW], wa1[OBW * AS], xb1[RW];
    // the remainder chunk of SPLIT_WX meets only the hi weights (lo x lo is below the
    // weights' own 22-bit representation)
    const int np = (SPLIT == SPLIT_WX && ch == 1) ? 1 : AS;
    auto fetch = [&](int it, u32x4 (&wa)[OBW * AS], u32x4 (&xb)[RW]) {
      const int tap = it / NCG, cg = it - tap * NCG;
      const int dy = tap / 3, dx = tap - 3 * dy;
      const u32x4* wp = wbase + tap * wstride_tap + (size_t)cg * wobtot * 64;
#pragma unroll
      for (int ob = 0; ob < OBW; ++ob)
#pragma unroll
        for (int part = 0; part < AS; ++part)
          if (part < np) wa[ob * AS + part] = wp[(ob * AS + part) * 64];
#pragma unroll
      for (int pb = 0; pb < RW; ++pb) xb[pb] = ldu4(tbase + ((pb + dy) * (kTW + 2) + dx) * LDP + KG * cg);
    };
    auto mma = [&](const u32x4 (&wa)[OBW * AS], const u32x4 (&xb)[RW]) {
#pragma unroll
      for (int pb = 0; pb < RW; ++pb)
#pragma unroll
        for (int ob = 0; ob < OBW; ++ob)
#pragma unroll
          for (int part = 0; part < AS; ++part)
            if (part < np) acc[pb][ob] = Mma<TC>::step(wa[ob * AS + part], xb[pb], acc[pb][ob]);
    };
    if constexpr (std::is_same<TC, float>::value) {
      // float: four MFMAs per fragment pair leave the loads enough time to land, and
      // the unrolled form (the copies fold into register renaming) schedules best
      fetch(0, wa0, xb0);
#pragma unroll 3
      for (int it = 0; it < NIT; ++it) {
        if (it + 1 < NIT) fetch(it + 1, wa1, xb1);
        mma(wa0, xb0);
        if (it + 1 < NIT) {
#pragma unroll
          for (int ob = 0; ob < OBW * AS; ++ob) wa0[ob] = wa1[ob];
#pragma unroll
          for (int pb = 0; pb < RW; ++pb) xb0[pb] = xb1[pb];
        }
      }
    } else {
      // 16-bit: one MFMA per fragment pair is too short to cover an L2 hit, so the
      // steps are unrolled and the A fragments (global) are requested PW steps ahead,
      // the B fragments (LDS) one step ahead.  The scheduling barrier after each step
      // keeps the compiler from hoisting every load to the top (which would cost far
      // more registers than the prefetch depth needs).
      constexpr int PW = 2;
      u32x4 wq[PW + 1][OBW * AS], xq[2][RW];
      auto fetch_w = [&](int it, u32x4 (&wa)[OBW * AS]) {
        const int tap = it / NCG, cg = it - tap * NCG;
        const u32x4* wp = wbase + tap * wstride_tap + (size_t)cg * wobtot * 64;
#pragma unroll
        for (int ob = 0; ob < OBW; ++ob)
#pragma unroll
          for (int part = 0; part < AS; ++part)
            if (part < np) wa[ob * AS + part] = wp[(ob * AS + part) * 64];
      };
      auto fetch_b = [&](int it, u32x4 (&xb)[RW]) {
        const int tap = it / NCG, cg = it - tap * NCG;
        const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
        for (int pb = 0; pb < RW; ++pb) xb[pb] = ldu4(tbase + ((pb + dy) * (kTW + 2) + dx) * LDP + KG * cg);
      };
#pragma unroll
      for (int k = 0; k < PW; ++k)
        if (k < NIT) fetch_w(k, wq[k]);
      fetch_b(0, xq[0]);
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        if (it + PW < NIT) fetch_w(it + PW, wq[(it + PW) % (PW + 1)]);
        if (it + 1 < NIT) fetch_b(it + 1, xq[(it + 1) & 1]);
        mma(wq[it % (PW + 1)], xq[it & 1]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  // a workgroup that holds all 64 output channels of its pixels: the results go through
  // the (now idle) LDS tile so that each wave stores whole pixels, one contiguous
  // kilobyte per instruction, instead of 32- or 64-byte pieces of sixteen pixels
  if constexpr (kStaged) {
    if (staged_rt) {
      if constexpr (kPre)
        conv_store_staged<TC, OBW, RW, PB, EPI, TC, true>(L, im, acc, ty0, tx0, wr, wo, tile, nullptr, resr);
      else
        conv_store_staged<TC, OBW, RW, PB, EPI>(L, im, acc, ty0, tx0, wr, wo, tile);
      return;
    }
  }
  // pixel shuffle with 64 high-resolution channels: a workgroup's eight row blocks are
  // two whole sub-pixels, written one at a time through LDS as whole pixels
  constexpr bool kStagedShuffle = std::is_same<TIN, TC>::value && std::is_same<TOUT, TC>::value && SPLIT == 0 &&
                                  NCHUNK == 1 && CCH == 64 && OB == 8 && EPI == EPI_SHUFFLE;
  if constexpr (kStagedShuffle) {
    if (L.ccout == 64 && obase % 4 == 0) {
      conv_store_shuffle_staged<TC, OBW, RW, PB>(L, im, acc, ty0, tx0, wr, wo, obase, tile);
      return;
    }
  }
  conv_store<TOUT, OBW, RW, EPI>(L, im, acc, ty0 + wr * RW, tx0, obase + wo * OBW, SPLIT ? L.oscale : nullptr);
  }
}

// 32x32x16 MFMA form of a bulk conv (16-bit maps, 64 input channels).  One MFMA takes
// 32 output channels x 32 pixels x 16 reduction indices: twice the work of a 16x16x32
// MFMA for the same 2 KB of operands, which halves the LDS and L1 bytes per flop.  The
// workgroup tile is 4 PB rows x 16 pixels as in conv_tile; wave w takes rows
// [w PB, (w+1) PB) as PB / 2 blocks of 32 pixels (two rows of 16: lane l's column is
// pixel l % 32 of the block, its quarter of K is channels 8 (l / 32) .. + 7 of the
// 16-channel group).  A fragments (L.wfrag = the 32-row packing, L.obtot counted in
// 32-row blocks) are requested two steps ahead, B fragments one step ahead.  Result
// register v of lane l is output channel 8 (v / 4) + 4 (l / 32) + v % 4 of its block.
template <typename TC, int OB32, int PB, int EPI>
__device__ __forceinline__ void conv_tile32(const ConvLayer& L, const ConvImg& im, int ty0, int tx0, int ob0,
                                            TC* tile) {
  static_assert(!std::is_same<TC, float>::value && !std::is_same<TC, f8>::value, "16-bit MFMA types");
  static_assert(PB == 2 || PB == 4, "whole 32-pixel blocks per wave");
  constexpr int CCH = 64, KG = 16, NCG = CCH / KG, NIT = 9 * NCG, RB = PB / 2, PW = 2;
  constexpr int LDP = ConvSmem<TC, CCH, PB>::LDP;
  typedef float f32x16 __attribute__((ext_vector_type(16)));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane & 31, h = lane >> 5;
  const int pr = p >> 4, pc = p & 15;

  const TC* src = static_cast<const TC*>(im.src0);
  if (im.sel != nullptr && *im.sel != 0u && im.alt0 != nullptr) src = static_cast<const TC*>(im.alt0);
  {
    constexpr int V = CCH / 8, NV = (4 * PB + 2) * (kTW + 2) * V, SB = 8;
    for (int i0 = 0; i0 < NV; i0 += SB * 256) {
      u32x4 rb[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 256 + (int)threadIdx.x;
        rb[u] = u32x4{0u, 0u, 0u, 0u};
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          const int ly = pix / (kTW + 2), lx = pix - ly * (kTW + 2);
          const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
          if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) rb[u] = ldu4(src + ((size_t)gy * im.W + gx) * CCH + 8 * v);
        }
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 256 + (int)threadIdx.x;
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          stu4(&tile[pix * LDP + 8 * v], rb[u]);
        }
      }
    }
  }
  __syncthreads();

  f32x16 acc[RB][OB32];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int ob = 0; ob < OB32; ++ob)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[rb][ob][v] = 0.0f;
  const u32x4* wbase = L.wfrag + (size_t)ob0 * 64 + lane;
  const TC* tbase = &tile[((wave * PB + pr) * (kTW + 2) + pc) * LDP + 8 * h];
  auto fetch_w = [&](int it, u32x4 (&wa)[OB32]) {
#pragma unroll
    for (int ob = 0; ob < OB32; ++ob) wa[ob] = wbase[((size_t)it * L.obtot + ob) * 64];
  };
  auto fetch_b = [&](int it, u32x4 (&xb)[RB]) {
    const int tap = it / NCG, cg = it - tap * NCG;
    const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) xb[rb] = ldu4(tbase + ((2 * rb + dy) * (kTW + 2) + dx) * LDP + KG * cg);
  };
  u32x4 wq[PW + 1][OB32], xq[2][RB];
#pragma unroll
  for (int k = 0; k < PW; ++k) fetch_w(k, wq[k]);
  fetch_b(0, xq[0]);
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    if (it + PW < NIT) fetch_w(it + PW, wq[(it + PW) % (PW + 1)]);
    if (it + 1 < NIT) fetch_b(it + 1, xq[(it + 1) & 1]);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int ob = 0; ob < OB32; ++ob) {
        if constexpr (std::is_same<TC, f16>::value)
          acc[rb][ob] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, wq[it % (PW + 1)][ob]),
                                                               __builtin_bit_cast(f16x8, xq[it & 1][rb]),
                                                               acc[rb][ob], 0, 0, 0);
        else
          acc[rb][ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, wq[it % (PW + 1)][ob]),
                                                                __builtin_bit_cast(bf16x8, xq[it & 1][rb]),
                                                                acc[rb][ob], 0, 0, 0);
      }
    __builtin_amdgcn_sched_barrier(0);
  }

  // epilogue: the same per-channel arithmetic as conv_store, four channels at a time
  TC* dst = static_cast<TC*>(im.dst);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int gy = ty0 + wave * PB + 2 * rb + pr, gx = tx0 + pc;
    if (gy >= im.H || gx >= im.W) continue;
#pragma unroll
    for (int ob = 0; ob < OB32; ++ob)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int row = (ob0 + ob) * 32 + 8 * m + 4 * h;     // A row = packed output row
        f32x4 v = f32x4{acc[rb][ob][4 * m], acc[rb][ob][4 * m + 1], acc[rb][ob][4 * m + 2], acc[rb][ob][4 * m + 3]};
        v += ld4(L.bias + row);
        if (EPI == EPI_LRELU) {
          store4f<TC>(dst + ((size_t)gy * im.W + gx) * L.ldy + row, lrelu4(v));
        } else if (EPI == EPI_RES) {
          const size_t at = ((size_t)gy * im.W + gx) * L.ldy + row;
          v += load4f<TC>(static_cast<const TC*>(im.res) + at);
          store4f<TC>(dst + at, v);
        } else {  // EPI_SHUFFLE: A row 16*g + t is channel 16*(g % NB) + t at sub-pixel g / NB
          const int g = row >> 4, nb = L.ccout >> 4, sp = g / nb, c = 16 * (g - sp * nb) + (row & 15);
          const int Y = L.sv * gy + sp / L.sh, X = L.sh * gx + sp % L.sh;
          store4f<TC>(dst + ((size_t)Y * (L.sh * im.W) + X) * L.ccout + c, lrelu4(v));
        }
      }
  }
}

template <typename TC, int OB32, int PB, int EPI>
__global__ __launch_bounds__(256) void k_conv32(ConvLayer L, ConvImg im) {
  __shared__ __attribute__((aligned(16))) TC tile[ConvSmem<TC, 64, PB>::N];
  const int tiles_x = (im.W + kTW - 1) / kTW;
  const int nobg = L.obtot / OB32;
  const int ntile = tiles_x * ((im.H + 4 * PB - 1) / (4 * PB));
  const int b = xcd_tile(blockIdx.x, ntile * nobg);
  const int t = b / nobg, obg = b - t * nobg;
  conv_tile32<TC, OB32, PB, EPI>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, obg * OB32, tile);
}

template <typename TC, int OB32, int PB, int EPI>
__global__ __launch_bounds__(256) void k_conv32_batch(ConvLayer L, const ConvImg* __restrict__ jobs,
                                                      const int* __restrict__ count) {
  __shared__ __attribute__((aligned(16))) TC tile[ConvSmem<TC, 64, PB>::N];
  const int njobs = count[0], total = count[1];
  const int nobg = L.obtot / OB32;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const ConvImg im = jobs[find_job(jobs, njobs, item)];
    const int local = item - im.item_begin;
    const int t = local / nobg, obg = local - t * nobg;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    conv_tile32<TC, OB32, PB, EPI>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, obg * OB32, tile);
    __syncthreads();
  }
}

template <typename TIN, typename TC, typename TOUT, int CCH, int NCHUNK, int OB, int PB, int EPI, int SPLIT, int WO>
__global__ __launch_bounds__(256) void k_conv3x3(ConvLayer L, ConvImg im) {
  __shared__ __attribute__((aligned(16))) TC tile[ConvSmem<TC, CCH, PB>::N];
  // block = (tile, output-block group), group fastest: the groups of a tile run next to
  // each other on one XCD and read its input from that XCD's L2
  const int tiles_x = (im.W + kTW - 1) / kTW;
  const int nobg = L.obtot / OB;
  const int ntile = tiles_x * ((im.H + 4 * PB - 1) / (4 * PB));
  const int b = xcd_tile(blockIdx.x, ntile * nobg);
  const int t = b / nobg, obg = b - t * nobg;
  conv_tile<TIN, TC, TOUT, CCH, NCHUNK, OB, PB, EPI, SPLIT, WO>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW,
                                                                 obg * OB, tile);
}

// Persistent form: item = (tile, output-block group) of one image of the job table.
template <typename TIN, typename TC, typename TOUT, int CCH, int NCHUNK, int OB, int PB, int EPI, int SPLIT, int WO>
__global__ __launch_bounds__(256) void k_conv3x3_batch(ConvLayer L, const ConvImg* __restrict__ jobs,
                                                       const int* __restrict__ count) {
  __shared__ __attribute__((aligned(16))) TC tile[ConvSmem<TC, CCH, PB>::N];
  const int njobs = count[0], total = count[1];
  const int nobg = L.obtot / OB;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const ConvImg im = jobs[find_job(jobs, njobs, item)];
    const int local = item - im.item_begin;
    const int t = local / nobg, obg = local - t * nobg;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    conv_tile<TIN, TC, TOUT, CCH, NCHUNK, OB, PB, EPI, SPLIT, WO>(L, im, (t / tiles_x) * 4 * PB,
                                                                   (t % tiles_x) * kTW, obg * OB, tile);
    __syncthreads();
  }
}

// ---- residual block as one kernel (16-bit maps, C = 64) ----
// A workgroup of eight waves produces a 16 x 16 tile of y = x + conv_b(LReLU(conv_a(x))).
// It stages x over the tile and a 2-pixel halo (20 x 20), computes the first conv over
// the tile and a 1-pixel halo (18 x 18 = 324 pixels, taken in 21 groups of 16 in
// row-major order, so the B operand's 16 pixels need not share a row) and keeps it in
// registers until every wave is done with the staged x, then writes it, LReLU-ed and
// rounded to the storage type, over the same LDS (zero outside the image: the second
// conv's zero padding), and runs the second conv over the tile; the skip is read from
// x in global memory.  Each output accumulates in the same order and rounds at the
// same points as the two separate launches, so the results are bit-identical to them.
// HBM traffic drops from ~5 map transfers per block to 2, for 21/16 of the first conv's
// MFMA work.
constexpr int kRbT = 16, kRbI = kRbT + 2, kRbX = kRbT + 4;
constexpr int kRbNI = kRbI * kRbI, kRbGA = (kRbNI + 15) / 16;

template <typename TC>
__global__ __launch_bounds__(512, 4) void k_resblock(ConvLayer La, ConvLayer Lb, ConvImg im) {
  constexpr int C = 64, LDP = C + 16 / (int)sizeof(TC);
  constexpr int KG = 32, QE = 8, NCG = 2, NIT = 9 * NCG, OB = 4, PW = 1;
  constexpr int NGA = (kRbGA + 7) / 8;            // first-conv pixel groups per wave, at most
  static_assert(kRbX * kRbX >= kRbNI, "the intermediate fits where x was staged");
  __shared__ __attribute__((aligned(16))) TC lds[kRbX * kRbX * LDP];

  const int tiles_x = (im.W + kRbT - 1) / kRbT;
  const int ntile = tiles_x * ((im.H + kRbT - 1) / kRbT);
  const int t = xcd_tile(blockIdx.x, ntile);
  const int ty0 = (t / tiles_x) * kRbT, tx0 = (t % tiles_x) * kRbT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const TC* x = static_cast<const TC*>(im.src0);
  TC* y = static_cast<TC*>(im.dst);

  // stage x over the tile and its 2-pixel halo (zero outside the image)
  {
    constexpr int V = C / 8, NV = kRbX * kRbX * V, SB = 4;
    for (int i0 = 0; i0 < NV; i0 += SB * 512) {
      u32x4 rb[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 512 + (int)threadIdx.x;
        rb[u] = u32x4{0u, 0u, 0u, 0u};
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          const int ly = pix / kRbX, lx = pix - ly * kRbX;
          const int gy = ty0 + ly - 2, gx = tx0 + lx - 2;
          if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) rb[u] = ldu4(x + ((size_t)gy * im.W + gx) * C + 8 * v);
        }
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int idx = i0 + u * 512 + (int)threadIdx.x;
        if (idx < NV) {
          const int pix = idx / V, v = idx - pix * V;
          stu4(&lds[pix * LDP + 8 * v], rb[u]);
        }
      }
    }
  }
  __syncthreads();

  // one conv over up to NGA pixel groups per wave: A and B fragments one step ahead,
  // every step unrolled with a scheduling barrier (registers are kept to 128 so that two
  // workgroups share a CU)
  auto conv = [&](const ConvLayer& L, const int (&pbase)[NGA], int ng, int row_stride, f32x4 (&acc)[NGA][OB]) {
    const u32x4* wbase = L.wfrag + lane;
    auto fetch_w = [&](int it, u32x4 (&wa)[OB]) {
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) wa[ob] = wbase[((size_t)it * L.obtot + ob) * 64];
    };
    auto fetch_b = [&](int it, u32x4 (&xb)[NGA]) {
      const int tap = it / NCG, cg = it - tap * NCG;
      const int dy = tap / 3, dx = tap - 3 * dy;
      const int off = (dy * row_stride + dx) * LDP + KG * cg;
#pragma unroll
      for (int k = 0; k < NGA; ++k) xb[k] = ldu4(&lds[pbase[k] + off]);
    };
#pragma unroll
    for (int k = 0; k < NGA; ++k)
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) acc[k][ob] = zero4();
    u32x4 wq[PW + 1][OB], xq[2][NGA];
#pragma unroll
    for (int k = 0; k < PW; ++k) fetch_w(k, wq[k]);
    fetch_b(0, xq[0]);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      if (it + PW < NIT) fetch_w(it + PW, wq[(it + PW) % (PW + 1)]);
      if (it + 1 < NIT) fetch_b(it + 1, xq[(it + 1) & 1]);
#pragma unroll
      for (int k = 0; k < NGA; ++k)
        if (k < ng)
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) acc[k][ob] = Mma<TC>::step(wq[it % (PW + 1)][ob], xq[it & 1][k], acc[k][ob]);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // first conv: groups wave, wave + 8, wave + 16 of the 324 intermediate pixels
  const int nga = (kRbGA - wave + 7) / 8;
  int pa[NGA];
#pragma unroll
  for (int k = 0; k < NGA; ++k) {
    const int i = min(16 * (wave + 8 * k) + j, kRbNI - 1);
    const int iy = i / kRbI, ix = i - iy * kRbI;
    pa[k] = (iy * kRbX + ix) * LDP + QE * q;
  }
  f32x4 acc[NGA][OB];
  conv(La, pa, nga, kRbX, acc);
  __syncthreads();   // every wave is done reading x from LDS
#pragma unroll
  for (int k = 0; k < NGA; ++k) {
    const int i = 16 * (wave + 8 * k) + j;
    if (k >= nga || i >= kRbNI) continue;
    const int iy = i / kRbI, ix = i - iy * kRbI;
    const int gy = ty0 - 1 + iy, gx = tx0 - 1 + ix;
    const bool inside = gy >= 0 && gy < im.H && gx >= 0 && gx < im.W;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = ob * 16 + 4 * q;
      f32x4 v = acc[k][ob];
      v += ld4(La.bias + row);
      store4f<TC>(&lds[i * LDP + row], inside ? lrelu4(v) : zero4());
    }
  }
  __syncthreads();

  // second conv: output rows 2 wave, 2 wave + 1 of the tile
  int pbb[NGA];
#pragma unroll
  for (int k = 0; k < NGA; ++k) pbb[k] = ((2 * wave + min(k, 1)) * kRbI + j) * LDP + QE * q;
  conv(Lb, pbb, 2, kRbI, acc);
#pragma unroll
  for (int pb = 0; pb < 2; ++pb) {
    const int gy = ty0 + 2 * wave + pb, gx = tx0 + j;
    if (gy >= im.H || gx >= im.W) continue;
    const size_t at = ((size_t)gy * im.W + gx) * C;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = ob * 16 + 4 * q;
      f32x4 v = acc[pb][ob];
      v += ld4(Lb.bias + row);
      v += load4f<TC>(x + at + row);
      store4f<TC>(y + at + row, v);
    }
  }
}

// ---- bulk conv with LDS-resident weights (16-bit and FP8 MFMA types) ----
// Switched off: its first launch on the device stopped in the HIP runtime ("cannot find
// symbol" for the kernel, 99.6 KB of static LDS, below the device's 160 KB) and no cause
// has been found in this code; the dispatch refuses these tiles and the tuner does not
// offer them until one is.
constexpr bool kLdsWeightTiles = false;

// A persistent workgroup owns one group of 64 output channels (4 output blocks) for all
// of its tiles: it copies that group's A fragments into LDS once, then for each tile
// reads both MFMA operands from LDS.  While the MFMAs of tile n run, the input of tile
// n+1 is already being loaded into registers (the step loop waits on LDS only, so these
// global loads stay in flight), and is written to the LDS tile after tile n's epilogue.
// Each wave computes PB rows x 16 pixels x 64 channels of the tile.
template <typename TC, int PB>
struct LwShape {
  static constexpr int OB = 4;
  static constexpr bool F8 = std::is_same<TC, f8>::value;
  static constexpr int NSTEP = F8 ? 5 : 18;                       // MFMA steps over 9 taps x 64 ch
  static constexpr int FB = F8 ? 32 : 16;                         // fragment bytes per lane
  static constexpr int WBYTES = NSTEP * OB * 64 * FB;
  static constexpr int LDP = ConvSmem<TC, 64, PB>::LDP;           // tile pixel stride (elements)
  static constexpr int TBYTES = ConvSmem<TC, 64, PB>::N * (int)sizeof(TC);
  static constexpr int NV = (4 * PB + 2) * (kTW + 2) * 8;          // 8-channel vectors per tile
  static constexpr int NR = (NV + 255) / 256;                      // per thread
  static constexpr int WG_PER_CU = 163840 / (WBYTES + TBYTES);
};

// The tile's input vectors of this thread (8 channels each), loaded into registers.
template <typename TC, int PB>
__device__ __forceinline__ void lw_load(const ConvImg& im, int ty0, int tx0, Raw8<f16>* rb, const void* src_v) {
  using S = LwShape<TC, PB>;
  const f16* src = static_cast<const f16*>(src_v);
#pragma unroll
  for (int u = 0; u < S::NR; ++u) {
    const int idx = u * 256 + (int)threadIdx.x;
    rb[u].zero();
    if (idx < S::NV) {
      const int pix = idx >> 3, v = idx & 7;
      const int ly = pix / (kTW + 2), lx = pix - ly * (kTW + 2);
      const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
      if (gy >= 0 && gy < im.H && gx >= 0 && gx < im.W) rb[u].load(src + ((size_t)gy * im.W + gx) * 64 + 8 * v);
    }
  }
}

template <typename TC, int PB>
__device__ __forceinline__ void lw_store(TC* tile, const Raw8<f16>* rb, float ainv) {
  using S = LwShape<TC, PB>;
#pragma unroll
  for (int u = 0; u < S::NR; ++u) {
    const int idx = u * 256 + (int)threadIdx.x;
    if (idx < S::NV) {
      const int pix = idx >> 3, v = idx & 7;
      TC* d = &tile[pix * S::LDP + 8 * v];
      if constexpr (S::F8) {
        f32x4 lo, hi;
        rb[u].to_f32(lo, hi);
        *reinterpret_cast<u32x2*>(d) = u32x2{f8x4_pack(lo * ainv), f8x4_pack(hi * ainv)};
      } else {
        stu4(d, rb[u].v);
      }
    }
  }
}

// MFMAs of one tile: A fragments from the LDS weight block, B from the LDS tile.
template <typename TC, int PB>
__device__ __forceinline__ void lw_mma(const uint8_t* wl, const TC* tile, f32x4 (&acc)[PB][4]) {
  using S = LwShape<TC, PB>;
  using Frag = typename Mma<TC>::Frag;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const Frag* wfr = reinterpret_cast<const Frag*>(wl) + lane;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) acc[pb][ob] = zero4();
  // B fragment address of step st: float16 steps are (tap, 32-channel group), quarter
  // q at channel 8 q; FP8 steps pair taps, quarter q at tap 2 st + q / 2, channel 32 (q % 2)
  auto boff = [&](int st) {
    int tap, ch;
    if constexpr (S::F8) {
      tap = min(2 * st + (q >> 1), 8);
      ch = 32 * (q & 1);
    } else {
      tap = st >> 1;
      ch = 32 * (st & 1) + 8 * q;
    }
    const int dy = tap / 3, dx = tap - 3 * dy;
    return ((wave * PB + dy) * (kTW + 2) + j + dx) * S::LDP + ch;
  };
  Frag a0[4], b0[PB], a1[4], b1[PB];
  auto fetch = [&](int st, Frag (&a)[4], Frag (&b)[PB]) {
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) a[ob] = Mma<TC>::ld(wfr + (st * 4 + ob) * 64);
    const int o = boff(st);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) b[pb] = Mma<TC>::ld(tile + o + pb * (kTW + 2) * S::LDP);
  };
  auto mma = [&](const Frag (&a)[4], const Frag (&b)[PB]) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) acc[pb][ob] = Mma<TC>::step(a[ob], b[pb], acc[pb][ob]);
  };
  fetch(0, a0, b0);
#pragma unroll 1
  for (int st = 0; st < S::NSTEP; st += 2) {
    if (st + 1 < S::NSTEP) fetch(st + 1, a1, b1);
    mma(a0, b0);
    if (st + 1 < S::NSTEP) {
      if (st + 2 < S::NSTEP) fetch(st + 2, a0, b0);
      mma(a1, b1);
    }
  }
}

// Copies output group obg's fragments (all steps, 4 blocks) from the packed layer into
// LDS in (step, block, lane) order.
template <typename TC, int PB>
__device__ __forceinline__ void lw_weights(const ConvLayer& L, int obg, uint8_t* wl) {
  using S = LwShape<TC, PB>;
  const u32x4* g = reinterpret_cast<const u32x4*>(L.wfrag);
  constexpr int N16 = S::WBYTES / 16;                  // 16-byte pieces
  constexpr int P = S::FB / 16;                        // pieces per lane fragment
  for (int i = threadIdx.x; i < N16; i += 256) {
    const int part = i % P, f = i / P;                 // f = (st * 4 + ob) * 64 + lane
    const int lane = f & 63, sb = f >> 6, ob = sb & 3, st = sb >> 2;
    const size_t gi = (((size_t)st * L.obtot + obg * 4 + ob) * 64 + lane) * P + part;
    reinterpret_cast<u32x4*>(wl)[i] = g[gi];
  }
}

template <typename TC, int PB, int EPI>
__device__ __forceinline__ void lw_run(const ConvLayer& L, const ConvImg* im1, const ConvImg* jobs,
                                       const int* count, uint8_t* smem) {
  using S = LwShape<TC, PB>;
  // storage type of the maps: bfloat16 for bfloat16 MFMA, float16 otherwise
  using TO = typename std::conditional<std::is_same<TC, bf16>::value, bf16, f16>::type;
  uint8_t* wl = smem;
  TC* tile = reinterpret_cast<TC*>(smem + S::WBYTES);
  const int nobg = L.obtot / 4;
  const int obg = blockIdx.x % nobg;                   // gridDim.x is a multiple of nobg
  const int wave = threadIdx.x >> 6;
  const float ainv = S::F8 ? *L.ainv : 1.0f;
  const int njobs = jobs ? count[0] : 1;
  const int total = jobs ? count[1] : 0;
  // item -> (image, tile origin); returns false past the end
  auto locate = [&](int item, ConvImg& im, int& ty0, int& tx0) -> bool {
    int local;
    if (jobs) {
      if (item >= total) return false;
      im = jobs[find_job(jobs, njobs, item)];
      local = item - im.item_begin;
    } else {
      im = *im1;
      const int ntile = ((im.W + kTW - 1) / kTW) * ((im.H + 4 * PB - 1) / (4 * PB));
      if (item >= ntile * nobg) return false;
      local = item;
    }
    const int t = local / nobg;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    ty0 = (t / tiles_x) * 4 * PB;
    tx0 = (t % tiles_x) * kTW;
    return true;
  };
  auto src_of = [&](const ConvImg& im) -> const void* {
    return (im.sel != nullptr && *im.sel != 0u && im.alt0 != nullptr) ? im.alt0 : im.src0;
  };

  lw_weights<TC, PB>(L, obg, wl);
  ConvImg im;
  int ty0, tx0;
  int item = blockIdx.x;
  if (!locate(item, im, ty0, tx0)) return;             // uniform per workgroup
  Raw8<f16> rb[S::NR];
  lw_load<TC, PB>(im, ty0, tx0, rb, src_of(im));
  lw_store<TC, PB>(tile, rb, ainv);
  __syncthreads();
  for (;;) {
    ConvImg nim;
    int nty0 = 0, ntx0 = 0;
    const int next = item + gridDim.x;
    const bool more = locate(next, nim, nty0, ntx0);
    if (more) lw_load<TC, PB>(nim, nty0, ntx0, rb, src_of(nim));
    f32x4 acc[PB][4];
    lw_mma<TC, PB>(wl, tile, acc);
    conv_store<TO, 4, PB, EPI>(L, im, acc, ty0 + wave * PB, tx0, obg * 4, S::F8 ? L.oscale : nullptr);
    __syncthreads();                                   // every wave is done with the tile
    if (!more) break;
    lw_store<TC, PB>(tile, rb, ainv);
    __syncthreads();
    item = next;
    im = nim;
    ty0 = nty0;
    tx0 = ntx0;
  }
}

template <typename TC, int PB, int EPI>
__global__ __launch_bounds__(256) void k_conv_lw(ConvLayer L, ConvImg im) {
  using S = LwShape<TC, PB>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[S::WBYTES + S::TBYTES];
  lw_run<TC, PB, EPI>(L, &im, nullptr, nullptr, smem);
}

template <typename TC, int PB, int EPI>
__global__ __launch_bounds__(256) void k_conv_lw_batch(ConvLayer L, const ConvImg* __restrict__ jobs,
                                                       const int* __restrict__ count) {
  using S = LwShape<TC, PB>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[S::WBYTES + S::TBYTES];
  lw_run<TC, PB, EPI>(L, nullptr, jobs, count, smem);
}

// ---- first conv 3 -> C on the vector ALUs: planar float RGB in, NHWC out, LReLU ----
// blockIdx.y selects 16 output channels, so every weight read is uniform (scalar loads).
template <typename TOUT>
__device__ __forceinline__ void conv_in_px(const float* __restrict__ rgb, const float* __restrict__ w,
                                           const float* __restrict__ b, int H, int W, int p, int o0,
                                           float (&out)[16]) {
  const int pc = min(p, H * W - 1);
  const int y = pc / W, x = pc - y * W;
  const size_t plane = (size_t)H * W;
  float in[27];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int yy = y + ky - 1, xx = x + kx - 1;
        in[c * 9 + ky * 3 + kx] =
            (yy >= 0 && yy < H && xx >= 0 && xx < W) ? rgb[c * plane + (size_t)yy * W + xx] : 0.0f;
      }
#pragma unroll
  for (int o = 0; o < 16; ++o) {
    float s = b[o0 + o];
    const float* wo = w + (size_t)(o0 + o) * 27;
#pragma unroll
    for (int k = 0; k < 27; ++k) s = fmaf(wo[k], in[k], s);
    out[o] = lrelu(s);
  }
}

// One workgroup: 4096 / C consecutive pixels (in row-major order) x all C channels.
// Thread t computes channel block t / PPW (16 channels) of pixel t % PPW, so the C/16
// waves of a pixel run share its inputs in L1; the results go through LDS and leave as
// one contiguous run of whole pixels.
template <typename TOUT, int C>
__device__ __forceinline__ void conv_in_block(const float* __restrict__ rgb, const float* __restrict__ w,
                                              const float* __restrict__ b, TOUT* __restrict__ dst, int H,
                                              int W, int blk, TOUT* lds) {
  constexpr int PPW = 256 / (C / 16), OLDP = C + 16 / (int)sizeof(TOUT);
  constexpr int E = 16 / (int)sizeof(TOUT), NPC = C / E;
  // the channel block is the same across a wave (PPW is a multiple of 64): scalar weights
  const int cb = __builtin_amdgcn_readfirstlane((int)threadIdx.x / PPW), pl = threadIdx.x - cb * PPW;
  const int p0 = blk * PPW;
  float out[16];
  conv_in_px<TOUT>(rgb, w, b, H, W, p0 + pl, 16 * cb, out);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    store4f<TOUT>(&lds[pl * OLDP + 16 * cb + 4 * v], f32x4{out[4 * v], out[4 * v + 1], out[4 * v + 2], out[4 * v + 3]});
  __syncthreads();
  const int np = min(PPW, H * W - p0);
#pragma unroll
  for (int idx = (int)threadIdx.x; idx < PPW * NPC; idx += 256) {
    const int px = idx / NPC, ck = idx - px * NPC;
    if (px < np) stu4(dst + (size_t)(p0 + px) * C + E * ck, ldu4(&lds[px * OLDP + E * ck]));
  }
}

template <typename TOUT, int C>
__global__ __launch_bounds__(256) void k_conv_in(const float* __restrict__ rgb, const float* __restrict__ w,
                                                 const float* __restrict__ b, TOUT* __restrict__ dst, int H, int W) {
  __shared__ __attribute__((aligned(16))) TOUT lds[(256 / (C / 16)) * (C + 16 / sizeof(TOUT))];
  conv_in_block<TOUT, C>(rgb, w, b, dst, H, W, blockIdx.x, lds);
}

// Persistent form: item = pixel run of one image.
template <typename TOUT, int C>
__global__ __launch_bounds__(256) void k_conv_in_batch(const float* __restrict__ w, const float* __restrict__ b,
                                                       const ConvInImg* __restrict__ jobs,
                                                       const int* __restrict__ count) {
  __shared__ __attribute__((aligned(16))) TOUT lds[(256 / (C / 16)) * (C + 16 / sizeof(TOUT))];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const ConvInImg& im = jobs[find_job(jobs, njobs, item)];
    conv_in_block<TOUT, C>(im.rgb, w, b, static_cast<TOUT*>(im.dst), im.H, im.W, item - im.item_begin, lds);
    __syncthreads();
  }
}

// ---- HR conv C -> 3 plus the bilinear x2 base, planar float RGB out ----
// The thin output conv is computed as "tap responses": R[3*tap + o][p] =
// sum_c w[o][c][tap] U[c][p] is a 27-row (padded to 32) by C product on MFMA, taken over
// every pixel of a 16x16 output tile and its one-pixel halo and kept in LDS; each
// output pixel then sums the nine responses of its shifted neighbours:
//   out[o][p] = b[o] + sum_tap R[3*tap + o][p + delta_tap] + base[o][p].
// Pixels outside the map have U = 0, hence R = 0: the conv's zero padding.
// tsel: 0 -> base of frame a, 1 -> frame b, 2 -> the mean of both.  The base is the
// bilinear resize by sv rows and sh columns (a factor of 1 keeps the axis; a factor of 2
// takes 3/4 of the nearest and 1/4 of the next sample along it, rows first).
__device__ __forceinline__ float up_sample(const float* pl, int H, int W, int Y, int X, int sv, int sh) {
  const int i = sv == 2 ? Y >> 1 : Y, jx = sh == 2 ? X >> 1 : X;
  const int i2 = (Y & 1) ? min(i + 1, H - 1) : max(i - 1, 0);
  const int j2 = (X & 1) ? min(jx + 1, W - 1) : max(jx - 1, 0);
  if (sv == 2 && sh == 2) {
    const float r0 = 0.75f * pl[(size_t)i * W + jx] + 0.25f * pl[(size_t)i2 * W + jx];
    const float r1 = 0.75f * pl[(size_t)i * W + j2] + 0.25f * pl[(size_t)i2 * W + j2];
    return 0.75f * r0 + 0.25f * r1;
  }
  if (sv == 2) return 0.75f * pl[(size_t)i * W + jx] + 0.25f * pl[(size_t)i2 * W + jx];
  if (sh == 2) return 0.75f * pl[(size_t)i * W + jx] + 0.25f * pl[(size_t)i * W + j2];
  return pl[(size_t)i * W + jx];
}

struct HrLayer {
  const u32x4* wfrag;    // [C/KG][2][64] fragments of the 32 x C response matrix
  const float* bias;     // [3]
};

constexpr int kHrT = 16, kHrRW = kHrT + 2, kHrNP = kHrRW * kHrRW, kHrNPB = (kHrNP + 15) / 16;
// R's row stride (floats): the 27 used response rows of a pixel, plus one for float maps.
// An odd stride puts the column reads of the sums below in distinct banks; 16-bit maps
// then fit four workgroups per CU (float maps measured faster at three).
template <typename TU>
constexpr int hr_ldr() {
  return sizeof(TU) == 2 ? 27 : 33;
}

template <typename TU, int C>
__device__ __forceinline__ void hr_tile(const HrLayer& L, const HrImg& im, int ty0, int tx0, float* R) {
  constexpr int T = kHrT, RW = kHrRW, NP = kHrNP, NPB = kHrNPB, LDR = hr_ldr<TU>();
  constexpr int KG = Mma<TU>::KG, QE = KG / 4, NCG = C / KG;
  const int H2 = im.sv * im.H, W2 = im.sh * im.W;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const TU* u = static_cast<const TU*>(im.u);

  u32x4 wa[NCG][2];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    wa[cg][0] = L.wfrag[(cg * 2 + 0) * 64 + lane];
    wa[cg][1] = L.wfrag[(cg * 2 + 1) * 64 + lane];
  }
  const u32x4 zero = {0u, 0u, 0u, 0u};
  // a wave's pixel blocks are wave, wave + 4, ...: all of their loads are issued before
  // the first MFMA, so the blocks do not each wait on a round trip of their own
  constexpr int MAXB = (NPB + 3) / 4;
  u32x4 xb[MAXB][NCG];
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int p = (wave + 4 * k) * 16 + j;
    const int ry = p / RW, rx = p - ry * RW;
    const int Y = ty0 + ry - 1, X = tx0 + rx - 1;
    const bool ok = wave + 4 * k < NPB && p < NP && Y >= 0 && Y < H2 && X >= 0 && X < W2;
    const TU* up = u + ((size_t)(ok ? Y : 0) * W2 + (ok ? X : 0)) * C + QE * q;
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) xb[k][cg] = ok ? ldu4(up + KG * cg) : zero;
  }
  // this thread's output pixel and its bilinear base; for 16-bit maps the base is
  // requested together with the tile's loads (both round trips overlap), for float maps
  // (twice the registers in flight) after the responses
  const int ly = threadIdx.x / T, lx = threadIdx.x - ly * T;
  const int Y = ty0 + ly, X = tx0 + lx;
  const bool out = Y < H2 && X < W2;
  const size_t lpl = (size_t)im.H * im.W, hpl = (size_t)H2 * W2;
  float base[3] = {0.0f, 0.0f, 0.0f};
  auto base_at = [&] {
    const float* rb = (im.sel != nullptr && *im.sel != 0u) ? im.rgb_a : im.rgb_b;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (im.tsel == 0) base[c] = up_sample(im.rgb_a + c * lpl, im.H, im.W, Y, X, im.sv, im.sh);
      else if (im.tsel == 1) base[c] = up_sample(rb + c * lpl, im.H, im.W, Y, X, im.sv, im.sh);
      else
        base[c] = 0.5f * (up_sample(im.rgb_a + c * lpl, im.H, im.W, Y, X, im.sv, im.sh) +
                          up_sample(rb + c * lpl, im.H, im.W, Y, X, im.sv, im.sh));
    }
  };
  constexpr bool kEarlyBase = sizeof(TU) == 2;
  if (kEarlyBase && out) base_at();
#pragma unroll
  for (int k = 0; k < MAXB; ++k) {
    const int pbk = wave + 4 * k;
    if (pbk >= NPB) continue;
    const int p = pbk * 16 + j;
    f32x4 acc0 = zero4(), acc1 = zero4();
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      acc0 = Mma<TU>::step(wa[cg][0], xb[k][cg], acc0);
      acc1 = Mma<TU>::step(wa[cg][1], xb[k][cg], acc1);
    }
    float* rp = &R[p * LDR];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rp[4 * q + r] = acc0[r];
      // rows 27 .. 31 are padding (written where the stride leaves room for them)
      if (LDR > 31 || 16 + 4 * q + r < 27) rp[16 + 4 * q + r] = acc1[r];
    }
  }
  __syncthreads();
  if (!out) return;
  if (!kEarlyBase) base_at();
  float s0 = L.bias[0], s1 = L.bias[1], s2 = L.bias[2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap - 3 * dy;
    const float* rp = &R[((ly + dy) * RW + lx + dx) * LDR + 3 * tap];
    s0 += rp[0];
    s1 += rp[1];
    s2 += rp[2];
  }
  im.dst[(size_t)Y * W2 + X] = s0 + base[0];
  im.dst[hpl + (size_t)Y * W2 + X] = s1 + base[1];
  im.dst[2 * hpl + (size_t)Y * W2 + X] = s2 + base[2];
}

template <typename TU, int C>
__global__ __launch_bounds__(256) void k_hr(HrLayer L, HrImg im) {
  __shared__ float R[kHrNPB * 16 * hr_ldr<TU>()];
  const int tiles_x = (im.sh * im.W + kHrT - 1) / kHrT;
  const int ntile = tiles_x * ((im.sv * im.H + kHrT - 1) / kHrT);
  const int t = xcd_tile(blockIdx.x, ntile);
  hr_tile<TU, C>(L, im, (t / tiles_x) * kHrT, (t % tiles_x) * kHrT, R);
}

template <typename TU, int C>
__global__ __launch_bounds__(256) void k_hr_batch(HrLayer L, const HrImg* __restrict__ jobs,
                                                  const int* __restrict__ count) {
  __shared__ float R[kHrNPB * 16 * hr_ldr<TU>()];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const HrImg im = jobs[find_job(jobs, njobs, item)];
    const int t = item - im.item_begin;
    const int tiles_x = (im.sh * im.W + kHrT - 1) / kHrT;
    hr_tile<TU, C>(L, im, (t / tiles_x) * kHrT, (t % tiles_x) * kHrT, R);
    __syncthreads();
  }
}

// ---- FP8 calibration: running max |x| of a layer input, and the scales derived from it ----

// amax_bits holds the running maximum as float bits (non-negative floats order like
// their bit patterns, so an unsigned atomic max is a float max).
template <typename T>
__global__ __launch_bounds__(256) void k_amax(const T* __restrict__ x, size_t n, uint32_t* amax_bits) {
  float m = 0.0f;
  for (size_t i = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4; i < n; i += (size_t)gridDim.x * 256 * 4) {
    if (i + 4 <= n) {
      const f32x4 v = load4f<T>(x + i);
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
    } else {
      for (size_t k = i; k < n; ++k) m = fmaxf(m, fabsf((float)x[k]));
    }
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  __shared__ float wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float b = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    atomicMax(amax_bits, __float_as_uint(b));
  }
}

// s_act = amax / 448 (1 when the layer has only seen zeros): ainv = 1 / s_act and
// oscale[r] = wscale[r] * s_act.
__global__ __launch_bounds__(256) void k_qscale(const uint32_t* __restrict__ amax_bits,
                                                const float* __restrict__ wscale, float* __restrict__ oscale,
                                                float* __restrict__ ainv, int rows) {
  const float a = __uint_as_float(*amax_bits);
  const float sa = a > 0.0f ? a / kF8Max : 1.0f;
  for (int r = threadIdx.x; r < rows; r += 256) oscale[r] = wscale[r] * sa;
  if (threadIdx.x == 0) *ainv = 1.0f / sa;
}

// ---------------------------------------------------------------- dispatch ----

// A launcher for one (types, shape, epilogue) instance, single image or batched.
struct ConvCall {
  const ConvLayer& L;
  const ConvImg* im;          // single image (by value into the kernel) ...
  const ConvImg* jobs;        // ... or a device job table with its count
  const int* count;
  hipStream_t s;
};

template <typename TIN, typename TC, typename TOUT, int CCH, int NCHUNK, int OB, int PB, int EPI, int SPLIT = 0,
          int WO = 1>
hipError_t run_conv(const ConvCall& c) {
  if (c.im) {
    const int ntile = ((c.im->W + kTW - 1) / kTW) * ((c.im->H + 4 * PB - 1) / (4 * PB));
    const dim3 grid(ntile * (c.L.obtot / OB));
    hipLaunchKernelGGL((k_conv3x3<TIN, TC, TOUT, CCH, NCHUNK, OB, PB, EPI, SPLIT, WO>), grid, dim3(256), 0, c.s,
                       c.L, *c.im);
  } else {
    hipLaunchKernelGGL((k_conv3x3_batch<TIN, TC, TOUT, CCH, NCHUNK, OB, PB, EPI, SPLIT, WO>), dim3(kBatchGrid),
                       dim3(256), 0, c.s, c.L, c.jobs, c.count);
  }
  return hipGetLastError();
}

// Storage type of a bulk conv whose MFMA type is T (FP8 layers keep float16 maps).
template <typename T>
struct Store {
  typedef T type;
};
template <>
struct Store<f8> {
  typedef f16 type;
};

template <typename T, int CCH, int PB, int WO>
hipError_t conv_bulk_pbw(const ConvCall& c, int epi) {
  typedef typename Store<T>::type S;
  switch (epi) {
    case EPI_LRELU:
      if (c.L.obtot % 4 == 0) return run_conv<S, T, S, CCH, 1, 4, PB, EPI_LRELU, SPLIT_NONE, WO>(c);
      return run_conv<S, T, S, CCH, 1, 2, PB, EPI_LRELU, SPLIT_NONE, WO>(c);
    case EPI_RES:
      if (c.L.obtot % 4 == 0) return run_conv<S, T, S, CCH, 1, 4, PB, EPI_RES, SPLIT_NONE, WO>(c);
      return run_conv<S, T, S, CCH, 1, 2, PB, EPI_RES, SPLIT_NONE, WO>(c);
    case EPI_SHUFFLE:
      // FP8 fragments are twice as wide: half the output blocks per workgroup; fewer
      // sub-pixels (a factor of 2 along one axis only) give fewer output blocks
      if constexpr (std::is_same<T, f8>::value) return run_conv<S, T, S, CCH, 1, 4, PB, EPI_SHUFFLE, SPLIT_NONE, WO>(c);
      else {
        if (c.L.obtot % 8 == 0) return run_conv<S, T, S, CCH, 1, 8, PB, EPI_SHUFFLE, SPLIT_NONE, WO>(c);
        if (c.L.obtot % 4 == 0) return run_conv<S, T, S, CCH, 1, 4, PB, EPI_SHUFFLE, SPLIT_NONE, WO>(c);
        return run_conv<S, T, S, CCH, 1, 2, PB, EPI_SHUFFLE, SPLIT_NONE, WO>(c);
      }
  }
  return hipErrorInvalidValue;
}

template <typename T, int CCH, int PB>
hipError_t conv_bulk_pb(const ConvCall& c, int epi, int wo) {
  if (wo == 1) return conv_bulk_pbw<T, CCH, PB, 1>(c, epi);
  // two waves along the output blocks
  if (wo == 2) return conv_bulk_pbw<T, CCH, PB, 2>(c, epi);
  return hipErrorInvalidValue;
}

template <typename TC, int PB, int EPI>
hipError_t run_lw(const ConvCall& c) {
  using S = LwShape<TC, PB>;
  if (c.L.obtot % 4 != 0) return hipErrorInvalidValue;
  const int nobg = c.L.obtot / 4;
  const int maxg = 256 * (S::WG_PER_CU > 0 ? S::WG_PER_CU : 1);
  if (c.im) {
    const int ntile = ((c.im->W + kTW - 1) / kTW) * ((c.im->H + 4 * PB - 1) / (4 * PB));
    int g = ntile * nobg < maxg ? ntile * nobg : maxg;
    g -= g % nobg;
    hipLaunchKernelGGL((k_conv_lw<TC, PB, EPI>), dim3(g), dim3(256), 0, c.s, c.L, *c.im);
  } else {
    hipLaunchKernelGGL((k_conv_lw_batch<TC, PB, EPI>), dim3(maxg), dim3(256), 0, c.s, c.L, c.jobs, c.count);
  }
  return hipGetLastError();
}

template <typename TC, int PB>
hipError_t conv_lw(const ConvCall& c, int epi) {
  switch (epi) {
    case EPI_LRELU: return run_lw<TC, PB, EPI_LRELU>(c);
    case EPI_RES: return run_lw<TC, PB, EPI_RES>(c);
    case EPI_SHUFFLE: return run_lw<TC, PB, EPI_SHUFFLE>(c);
  }
  return hipErrorInvalidValue;
}

// Largest static LDS a workgroup may use on the current device (queried once per device).
int device_lds_limit() {
  static int limit[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
  if (limit[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) v = 65536;
    limit[dev] = v;
  }
  return limit[dev];
}

template <typename T, int CCH>
int bulk_lds_bytes(int tile) {
  const int pb = tile_pb(tile);
  if (tile_lw(tile)) {
    if constexpr (!std::is_same<T, float>::value && CCH == 64) {
      if (pb == 2) return LwShape<T, 2>::WBYTES + LwShape<T, 2>::TBYTES;
      if (pb == 4) return LwShape<T, 4>::WBYTES + LwShape<T, 4>::TBYTES;
    }
    return 1 << 30;
  }
  const int th = 4 * pb;
  return (th + 2) * (kTW + 2) * (CCH + 16 / (int)sizeof(T)) * (int)sizeof(T);
}

// Residual-block convs and the pixel-shuffle conv: storage and MFMA in T; tile is a
// tile code (rows per wave, waves along the output blocks, LDS-resident weights).
// A tile whose LDS exceeds the device's per-workgroup limit is refused, not launched.
template <typename TC, int OB32, int PB, int EPI>
hipError_t run_conv32(const ConvCall& c) {
  if (c.L.obtot % OB32 != 0) return hipErrorInvalidValue;
  if (c.im) {
    const int ntile = ((c.im->W + kTW - 1) / kTW) * ((c.im->H + 4 * PB - 1) / (4 * PB));
    hipLaunchKernelGGL((k_conv32<TC, OB32, PB, EPI>), dim3(ntile * (c.L.obtot / OB32)), dim3(256), 0, c.s, c.L,
                       *c.im);
  } else {
    hipLaunchKernelGGL((k_conv32_batch<TC, OB32, PB, EPI>), dim3(kBatchGrid), dim3(256), 0, c.s, c.L, c.jobs,
                       c.count);
  }
  return hipGetLastError();
}

// 32x32 form: c.L carries the 32-row fragments with obtot in 32-row blocks.
template <typename TC, int PB>
hipError_t conv32_pb(const ConvCall& c, int epi) {
  switch (epi) {
    case EPI_LRELU: return run_conv32<TC, 2, PB, EPI_LRELU>(c);
    case EPI_RES: return run_conv32<TC, 2, PB, EPI_RES>(c);
    case EPI_SHUFFLE: return run_conv32<TC, PB == 2 ? 4 : 2, PB, EPI_SHUFFLE>(c);
  }
  return hipErrorInvalidValue;
}

template <typename T, int CCH>
hipError_t conv_bulk(const ConvCall& c, int epi, int tile) {
  const int pb = tile_pb(tile), wo = tile_wo(tile);
  if (bulk_lds_bytes<T, CCH>(tile) > device_lds_limit()) return hipErrorInvalidConfiguration;
  if (tile_lw(tile)) {
    if (!kLdsWeightTiles) return hipErrorNotSupported;
    if constexpr (!std::is_same<T, float>::value && CCH == 64) {
      if (pb == 2) return conv_lw<T, 2>(c, epi);
      if (pb == 4) return conv_lw<T, 4>(c, epi);
    }
    return hipErrorInvalidValue;
  }
  if (tile_m32(tile)) {
    if constexpr (!std::is_same<T, float>::value && !std::is_same<T, f8>::value && CCH == 64) {
      if (wo != 1) return hipErrorInvalidValue;
      if (pb == 2) return conv32_pb<T, 2>(c, epi);
      if (pb == 4) return conv32_pb<T, 4>(c, epi);
    }
    return hipErrorInvalidValue;
  }
  if (pb == 1) return conv_bulk_pb<T, CCH, 1>(c, epi, wo);
  if (pb == 2) return conv_bulk_pb<T, CCH, 2>(c, epi, wo);
  if (pb == 4) return conv_bulk_pb<T, CCH, 4>(c, epi, wo);
  return hipErrorInvalidValue;
}

// Offset head: first conv reads the two feature maps (TIN) and computes in float, on
// float MFMA or (split) on float16 MFMA with two-part weights.  The split form has
// three tile shapes (see head_ob): rows per wave 2 with all of a workgroup's output
// blocks per wave, rows per wave 4 with two output blocks, and two waves along the
// output blocks.
template <typename TIN, int CCH>
hipError_t conv_off1(const ConvCall& c, bool split, int tile) {
  const int pb = tile_pb(tile), wo = tile_wo(tile);
  if (split) {
    if constexpr (std::is_same<TIN, float>::value) return hipErrorInvalidValue;
    else {
      if (wo == 2 && pb == 2) {
        if (c.L.obtot % 4 == 0) return run_conv<TIN, f16, float, CCH, 2, 4, 2, EPI_LRELU, SPLIT_W, 2>(c);
        if (c.L.obtot % 2 == 0) return run_conv<TIN, f16, float, CCH, 2, 2, 2, EPI_LRELU, SPLIT_W, 2>(c);
        return hipErrorInvalidValue;
      }
      if (wo == 1 && pb == 4) return run_conv<TIN, f16, float, CCH, 2, 2, 4, EPI_LRELU, SPLIT_W>(c);
      if (wo != 1 || pb != 2) return hipErrorInvalidValue;
      if (c.L.obtot % 4 == 0) return run_conv<TIN, f16, float, CCH, 2, 4, 2, EPI_LRELU, SPLIT_W>(c);
      return run_conv<TIN, f16, float, CCH, 2, 2, 2, EPI_LRELU, SPLIT_W>(c);
    }
  }
  if (wo != 1 || pb != 2) return hipErrorInvalidValue;
  if (c.L.obtot % 4 == 0) return run_conv<TIN, float, float, CCH, 2, 4, 2, EPI_LRELU>(c);
  return run_conv<TIN, float, float, CCH, 2, 2, 2, EPI_LRELU>(c);
}

template <int CCH>
hipError_t conv_off2(const ConvCall& c, bool split, int tile) {
  const int pb = tile_pb(tile), wo = tile_wo(tile);
  if (split) {
    if (wo == 2 && pb == 2 && c.L.obtot % 2 == 0)
      return run_conv<float, f16, float, CCH, 2, 2, 2, EPI_OFFSET, SPLIT_WX, 2>(c);
    if (wo == 1 && pb == 4 && c.L.obtot % 2 == 0)
      return run_conv<float, f16, float, CCH, 2, 2, 4, EPI_OFFSET, SPLIT_WX>(c);
    if (wo != 1 || pb != 2) return hipErrorInvalidValue;
    if (c.L.obtot % 7 == 0) return run_conv<float, f16, float, CCH, 2, 7, 2, EPI_OFFSET, SPLIT_WX>(c);
    if (c.L.obtot % 4 == 0) return run_conv<float, f16, float, CCH, 2, 4, 2, EPI_OFFSET, SPLIT_WX>(c);
    return run_conv<float, f16, float, CCH, 2, 1, 2, EPI_OFFSET, SPLIT_WX>(c);
  }
  if (wo != 1 || pb != 2) return hipErrorInvalidValue;
  if (c.L.obtot % 7 == 0) return run_conv<float, float, float, CCH, 1, 7, 2, EPI_OFFSET>(c);
  if (c.L.obtot % 4 == 0) return run_conv<float, float, float, CCH, 1, 4, 2, EPI_OFFSET>(c);
  return run_conv<float, float, float, CCH, 1, 1, 2, EPI_OFFSET>(c);
}

template <typename T>
hipError_t conv_any(const ConvCall& c, int epi, int role, int cch, int pb, bool split) {
  if (role == CONV_OFF1) {
    if (cch == 64) return conv_off1<T, 64>(c, split, pb);
    if (cch == 32) return conv_off1<T, 32>(c, split, pb);
    return hipErrorInvalidValue;
  }
  if (cch == 64) return conv_bulk<T, 64>(c, epi, pb);
  if (cch == 32) return conv_bulk<T, 32>(c, epi, pb);
  return hipErrorInvalidValue;
}

hipError_t conv_dispatch(const PackedConv& P, int role, int epi, int tin, int pb, const ConvCall& c) {
  // offset head: float fragments, or two-part float16 fragments (split) with 1/s per row
  const bool split = (role == CONV_OFF1 || role == CONV_OFF2) && P.tc == DT_F16;
  if (split && !P.oscale) return hipErrorInvalidValue;
  if (role == CONV_OFF2) {
    if (tin != DT_F32 || (P.tc != DT_F32 && !split)) return hipErrorInvalidValue;
    const int cch = split ? P.cin / 2 : P.cin;   // split: packed over [hi | lo] chunks
    if (cch == 64) return conv_off2<64>(c, split, pb);
    if (cch == 32) return conv_off2<32>(c, split, pb);
    return hipErrorInvalidValue;
  }
  if (P.tc == DT_F8) {
    if (role != CONV_BULK || tin != DT_F16 || P.cin != 64 || !P.oscale || !P.ainv) return hipErrorInvalidValue;
    return conv_bulk<f8, 64>(c, epi, pb);
  }
  if (role == CONV_BULK && tile_m32(pb)) {
    if (!P.frag32 || P.tc != tin) return hipErrorInvalidValue;
    ConvLayer L32 = c.L;
    L32.wfrag = reinterpret_cast<const u32x4*>(P.frag32);
    L32.obtot = P.cout / 32;
    const ConvCall c32{L32, c.im, c.jobs, c.count, c.s};
    switch (tin) {
      case DT_F16: return conv_bulk<f16, 64>(c32, epi, pb);
      case DT_BF16: return conv_bulk<bf16, 64>(c32, epi, pb);
    }
    return hipErrorInvalidValue;
  }
  const int cch = role == CONV_OFF1 ? P.cin / 2 : P.cin;
  if (role == CONV_OFF1 && P.tc != DT_F32 && !split) return hipErrorInvalidValue;
  if (role != CONV_OFF1 && P.tc != tin) return hipErrorInvalidValue;
  switch (tin) {
    case DT_F32: return conv_any<float>(c, epi, role, cch, pb, split);
    case DT_F16: return conv_any<f16>(c, epi, role, cch, pb, split);
    case DT_BF16: return conv_any<bf16>(c, epi, role, cch, pb, split);
  }
  return hipErrorInvalidValue;
}

ConvLayer make_layer(const PackedConv& P, int ldy, int sig_lo) {
  ConvLayer L;
  L.wfrag = reinterpret_cast<const u32x4*>(P.frag);
  L.bias = P.bias;
  L.oscale = P.oscale;
  L.ainv = P.ainv;
  L.ldy = ldy;
  L.cout = P.cout;
  L.sig_lo = sig_lo;
  L.obtot = P.obtot;
  L.sv = P.sv;
  L.sh = P.sh;
  L.ccout = P.cout / (P.sv * P.sh);
  return L;
}

template <typename TU, int C>
void run_hr(const HrLayer& L, const HrImg* im, const HrImg* jobs, const int* count, hipStream_t s) {
  if (im) hipLaunchKernelGGL((k_hr<TU, C>), dim3(hr_items(im->H, im->W, im->sv, im->sh)), dim3(256), 0, s, L, *im);
  else hipLaunchKernelGGL((k_hr_batch<TU, C>), dim3(kBatchGrid), dim3(256), 0, s, L, jobs, count);
}

hipError_t hr_dispatch(const PackedConv& P, int tu, const HrImg* im, const HrImg* jobs, const int* count,
                       hipStream_t s) {
  if (P.tc != tu) return hipErrorInvalidValue;
  HrLayer L;
  L.wfrag = reinterpret_cast<const u32x4*>(P.frag);
  L.bias = P.bias;
  const int C = P.cin;
#define NV_HR(TU) (C == 64 ? (run_hr<TU, 64>(L, im, jobs, count, s), true) : C == 32 ? (run_hr<TU, 32>(L, im, jobs, count, s), true) : false)
  bool ok = false;
  if (tu == DT_F32) ok = NV_HR(float);
  else if (tu == DT_F16) ok = NV_HR(f16);
  else if (tu == DT_BF16) ok = NV_HR(bf16);
#undef NV_HR
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

}  // namespace

int conv_ob(int role, int epi, int obtot, int tc, int tile) {
  const bool split = tc == DT_F16;
  const int pb = tile_pb(tile), wo = tile_wo(tile);
  if (role == CONV_OFF2) {
    if (split && (wo == 2 || pb == 4)) return 2;
    return obtot % 7 == 0 ? 7 : (obtot % 4 == 0 ? 4 : 1);
  }
  if (role == CONV_OFF1) {
    if (split && pb == 4) return 2;
    return obtot % 4 == 0 ? 4 : 2;
  }
  if (tile_lw(tile)) return 4;
  if (tile_m32(tile)) return epi == EPI_SHUFFLE ? (pb == 2 ? 8 : 4) : 4;   // in 16-row blocks
  if (epi == EPI_SHUFFLE) return tc == DT_F8 ? 4 : (obtot % 8 == 0 ? 8 : (obtot % 4 == 0 ? 4 : 2));
  return obtot % 4 == 0 ? 4 : 2;
}

template <int C>
hipError_t launch_conv_in_c(const PlainConv& L, int tout, const float* rgb, void* dst, int H, int W, hipStream_t s) {
  const dim3 grid(conv_in_items(H, W, C));
  if (tout == DT_F32)
    hipLaunchKernelGGL((k_conv_in<float, C>), grid, dim3(256), 0, s, rgb, L.w, L.b, static_cast<float*>(dst), H, W);
  else if (tout == DT_F16)
    hipLaunchKernelGGL((k_conv_in<f16, C>), grid, dim3(256), 0, s, rgb, L.w, L.b, static_cast<f16*>(dst), H, W);
  else if (tout == DT_BF16)
    hipLaunchKernelGGL((k_conv_in<bf16, C>), grid, dim3(256), 0, s, rgb, L.w, L.b, static_cast<bf16*>(dst), H, W);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv_in(const PlainConv& L, int tout, const float* rgb, void* dst, int H, int W,
                          hipStream_t s) {
  if (L.cout == 64) return launch_conv_in_c<64>(L, tout, rgb, dst, H, W, s);
  if (L.cout == 32) return launch_conv_in_c<32>(L, tout, rgb, dst, H, W, s);
  return hipErrorInvalidValue;
}

template <int C>
hipError_t launch_conv_in_batch_c(const PlainConv& L, int tout, const ConvInImg* jobs, const int* count,
                                  hipStream_t s) {
  const dim3 grid(kBatchGrid);
  if (tout == DT_F32) hipLaunchKernelGGL((k_conv_in_batch<float, C>), grid, dim3(256), 0, s, L.w, L.b, jobs, count);
  else if (tout == DT_F16) hipLaunchKernelGGL((k_conv_in_batch<f16, C>), grid, dim3(256), 0, s, L.w, L.b, jobs, count);
  else if (tout == DT_BF16) hipLaunchKernelGGL((k_conv_in_batch<bf16, C>), grid, dim3(256), 0, s, L.w, L.b, jobs, count);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_conv_in_batch(const PlainConv& L, int tout, const ConvInImg* jobs, const int* count,
                                hipStream_t s) {
  if (L.cout == 64) return launch_conv_in_batch_c<64>(L, tout, jobs, count, s);
  if (L.cout == 32) return launch_conv_in_batch_c<32>(L, tout, jobs, count, s);
  return hipErrorInvalidValue;
}

int bulk_tile_lds(int tc, int cch, int tile) {
  if (cch != 32 && cch != 64) return 1 << 30;
  switch (tc) {
    case DT_F32: return cch == 64 ? bulk_lds_bytes<float, 64>(tile) : bulk_lds_bytes<float, 32>(tile);
    case DT_F16: return cch == 64 ? bulk_lds_bytes<f16, 64>(tile) : bulk_lds_bytes<f16, 32>(tile);
    case DT_BF16: return cch == 64 ? bulk_lds_bytes<bf16, 64>(tile) : bulk_lds_bytes<bf16, 32>(tile);
    case DT_F8: return bulk_lds_bytes<f8, 64>(tile);
  }
  return 1 << 30;
}

int lds_limit() { return device_lds_limit(); }

bool lds_weight_tiles() { return kLdsWeightTiles; }

hipError_t launch_conv(const PackedConv& P, int role, int epi, int tin, int pb, const ConvImg& im,
                       int ldy, int sig_lo, hipStream_t s) {
  const ConvLayer L = make_layer(P, ldy, sig_lo);
  const ConvCall c{L, &im, nullptr, nullptr, s};
  return conv_dispatch(P, role, epi, tin, pb, c);
}

bool resblock_supported(const PackedConv& A, const PackedConv& Bc, int tin) {
  return (tin == DT_F16 || tin == DT_BF16) && A.tc == tin && Bc.tc == tin && A.cin == 64 && A.cout == 64 &&
         Bc.cin == 64 && Bc.cout == 64 && A.obtot == 4 && Bc.obtot == 4;
}

hipError_t launch_resblock(const PackedConv& A, const PackedConv& Bc, int tin, const ConvImg& im, hipStream_t s) {
  if (!resblock_supported(A, Bc, tin) || im.src0 == im.dst) return hipErrorInvalidValue;
  const ConvLayer La = make_layer(A, 64, 0), Lb = make_layer(Bc, 64, 0);
  const int ntile = ((im.W + kRbT - 1) / kRbT) * ((im.H + kRbT - 1) / kRbT);
  if (tin == DT_F16) hipLaunchKernelGGL(k_resblock<f16>, dim3(ntile), dim3(512), 0, s, La, Lb, im);
  else hipLaunchKernelGGL(k_resblock<bf16>, dim3(ntile), dim3(512), 0, s, La, Lb, im);
  return hipGetLastError();
}

hipError_t launch_conv_batch(const PackedConv& P, int role, int epi, int tin, int pb,
                             const ConvImg* jobs, const int* count, int ldy, int sig_lo, hipStream_t s) {
  const ConvLayer L = make_layer(P, ldy, sig_lo);
  const ConvCall c{L, nullptr, jobs, count, s};
  return conv_dispatch(P, role, epi, tin, pb, c);
}

hipError_t launch_amax(int dt, const void* x, size_t n, uint32_t* amax_bits, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 4 * 256 - 1) / (4 * 256);
  const dim3 grid((unsigned)(blocks < 1024 ? blocks : 1024));
  if (dt == DT_F16) hipLaunchKernelGGL((k_amax<f16>), grid, dim3(256), 0, s, static_cast<const f16*>(x), n, amax_bits);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_amax<float>), grid, dim3(256), 0, s, static_cast<const float*>(x), n, amax_bits);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_qscale(const uint32_t* amax_bits, const float* wscale, float* oscale, float* ainv, int rows,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_qscale, dim3(1), dim3(256), 0, s, amax_bits, wscale, oscale, ainv, rows);
  return hipGetLastError();
}

hipError_t launch_hr(const PackedConv& P, int tu, const HrImg& im, hipStream_t s) {
  return hr_dispatch(P, tu, &im, nullptr, nullptr, s);
}

hipError_t launch_hr_batch(const PackedConv& P, int tu, const HrImg* jobs, const int* count, hipStream_t s) {
  return hr_dispatch(P, tu, nullptr, jobs, count, s);
}

}  // namespace nv

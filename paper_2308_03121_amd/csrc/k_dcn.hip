// The modulated deformable convolution of the fusion stage (gfx950): the bilinear
// samples of both feature maps at the offset positions, modulated by the masks, and their
// contraction with the weights on MFMA.  Activations are NHWC; a workgroup owns a tile of
// TH x 16 output pixels (TH = 4 waves x PB rows) and all C output channels.  In the MFMA
// the weights are the A operand (rows = output channels) and the samples the B operand
// (columns = the 16 pixels of one tile row), so each lane ends up holding four
// consecutive output channels of one pixel.
#include <type_traits>

#include "nv_internal.h"
#include "nv_mma.h"

namespace nv {
namespace {

// ---- modulated deformable conv, stride 1, pad 1, 3x3, over cat(fa, fb) ----
// Over a TH x 16 pixel tile, per phase (below):
//  gather: one work item per (pixel, channel chunk, tap) computes the sampling position
//          and the four bilinear weights (float), reads the chunk's channels at the four
//          corners (vectors of the NHWC maps), scales by the mask and writes the
//          modulated samples to LDS in the MFMA type;
//  MFMA:   the tile's samples times the phase's weights, accumulated over phases.
struct DcnLayer {
  const void* wfrag;        // fragments of the MFMA type
  const float* bias;
  const float* oscale;      // FP8: per output channel weight scale x activation scale
  const float* ainv;        // FP8: 1 / activation scale (device scalar)
  int ldo, groups, obtot;
};

// The reduction index K of the DCN (input channel ci of the concatenated pair, tap) is
// walked in phases.  The channels are cut into chunks of CW = min(CPG, KG) consecutive
// channels (CPG channels per offset group, KG channels per MFMA step group); a phase
// covers GP = KG / CW consecutive chunks with all nine taps, ordered (chunk, tap,
// channel), so a phase reads each of its sampling positions' offsets once and gathers
// its chunks' channels for all taps at once.  Every phase is 9 MFMA steps deep.
template <typename TC, int CPG>
struct DcnPhase {
  static constexpr int KG = Mma<TC>::KG;
  static constexpr int CW = CPG < KG ? CPG : KG;
  static constexpr int GP = KG / CW;
  static constexpr int NCH = CPG / CW;              // chunks per offset group
  static constexpr int K = 9 * KG;                  // K of one phase
  static constexpr int LDS_P = K + 16 / (int)sizeof(TC);
};

template <typename TC, int CPG, int PB>
struct DcnSmem {
  static constexpr int N = 4 * PB * kTW * DcnPhase<TC, CPG>::LDS_P;
};

// The DCN epilogue: bias, LReLU and the store of the tile's C output channels (through
// the idle LDS buffer S of NS elements for float and 16-bit maps, so that each wave
// stores whole pixels; FP8 outputs scaled per channel and stored directly).  A wave's
// accumulators acc[r][b] are pixel row wave * PB + r and channel block b, or with CS
// (channel split: one block of 16 channels per wave) pixel row r of the PB-row tile and
// channel block wave.
template <typename TF, typename TC, int C, int PB, int NS, bool CS = false, int OB = C / 16>
__device__ __forceinline__ void dcn_store(const DcnLayer& L, const DcnImg& im, int ty0, int tx0,
                                          const f32x4 (&acc)[PB][OB], TC* S) {
  constexpr int TH = CS ? PB : 4 * PB;
  static_assert(!CS || (OB == 1 && std::is_same<TF, TC>::value), "channel split: one block per wave, staged");
  constexpr bool kF8 = std::is_same<TC, f8>::value;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  TF* dst = static_cast<TF*>(im.dst);
  const int gx = tx0 + j;
  if constexpr (std::is_same<TF, TC>::value) {
    // through the idle sample buffer, so that each wave stores whole pixels (one
    // contiguous kilobyte per instruction); same arithmetic as the direct form
    constexpr int OLDP = C + 16 / (int)sizeof(TF);
    static_assert(TH * kTW * OLDP <= NS, "output tile fits the staging buffer");
    __syncthreads();
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int r = CS ? pb : wave * PB + pb;
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) {
        const int row = (CS ? wave : ob) * 16 + 4 * q;
        const f32x4 v = acc[pb][ob] + ld4(L.bias + row);
        store4f<TF>(&S[(r * kTW + j) * OLDP + row], lrelu4(v));
      }
    }
    __syncthreads();
    constexpr int E = 16 / (int)sizeof(TF), NPC = C / E;
#pragma unroll
    for (int idx = (int)threadIdx.x; idx < TH * kTW * NPC; idx += 256) {
      const int px = idx / NPC, ck = idx - px * NPC;
      const int oy = ty0 + px / kTW, ox = tx0 + px % kTW;
      if (oy < im.H && ox < im.W) stu4(dst + ((size_t)oy * im.W + ox) * C + E * ck, ldu4(&S[px * OLDP + E * ck]));
    }
    return;
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int gy = ty0 + wave * PB + pb;
    if (gy >= im.H || gx >= im.W) continue;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = ob * 16 + 4 * q;
      const f32x4 a = kF8 ? acc[pb][ob] * ld4(L.oscale + row) : acc[pb][ob];
      const f32x4 v = a + ld4(L.bias + row);
      store4f<TF>(dst + ((size_t)gy * im.W + gx) * C + row, lrelu4(v));
    }
  }
}

// Float samples in 16-channel chunks: the four 16-byte pieces of chunk c sit rotated by
// c / 2 inside the chunk, so that stores of consecutive taps (chunks 64 bytes apart) fall
// in eight different 16-byte bank groups.
template <typename TC, int CPG>
constexpr bool dcn_rot() {
  return std::is_same<TC, float>::value && DcnPhase<TC, CPG>::CW == 16;
}
template <bool ROT>
__device__ __forceinline__ int dcn_piece(int c, int v4) {
  return ROT ? ((v4 + (c >> 1)) & 3) : v4;
}

// The sampling position of one (pixel, tap) at integer base (by, bx) = pixel + tap - 1
// plus the offset (dy, dx): the top-left corner (y0, x0) and the four bilinear weights
// times the modulation m, zero for a corner outside the H x W map.  Positions are clamped
// to [-2, H + 1] x [-2, W + 1]: beyond one pixel outside the map every sample is zero, and
// the clamp keeps the integer conversion defined for any offset value.
__device__ __forceinline__ void dcn_corners(int by, int bx, float dy, float dx, float m, int H, int W, int& y0,
                                            int& x0, float (&cw)[4]) {
  const float py = fminf(fmaxf((float)by + dy, -2.0f), (float)H + 1.0f);
  const float px = fminf(fmaxf((float)bx + dx, -2.0f), (float)W + 1.0f);
  const float y0f = floorf(py), x0f = floorf(px);
  const float ly = py - y0f, lx = px - x0f;
  y0 = (int)y0f;
  x0 = (int)x0f;
  // a corner is inside when its row and its column are (each tested once)
  bool rok[2], cok[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    rok[k] = (unsigned)(y0 + k) < (unsigned)H;
    cok[k] = (unsigned)(x0 + k) < (unsigned)W;
  }
#pragma unroll
  for (int cy = 0; cy < 2; ++cy)
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
      cw[2 * cy + cx] = rok[cy] && cok[cx] ? (cy ? ly : 1.0f - ly) * (cx ? lx : 1.0f - lx) * m : 0.0f;
}

// The weighted sum of the four corners' CW channels (raw vectors of 8 channels), rounded
// to TC and stored at sp: chunk-contiguous, or rotated pieces (ROT) for chunk c.
template <typename TF, typename TC, int NV8, bool ROT>
__device__ __forceinline__ void dcn_blend_store(const Raw8<TF> (&raw)[4][NV8], const float (&cw)[4], TC* sp, int c) {
#pragma unroll
  for (int v = 0; v < NV8; ++v) {
    f32x4 lo = zero4(), hi = zero4();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      f32x4 a, b;
      raw[k][v].to_f32(a, b);
      lo += cw[k] * a;
      hi += cw[k] * b;
    }
    if constexpr (ROT) {
      store4f<TC>(sp + 4 * dcn_piece<ROT>(c, 2 * v), lo);
      store4f<TC>(sp + 4 * dcn_piece<ROT>(c, 2 * v + 1), hi);
    } else {
      store8f<TC>(sp + 8 * v, lo, hi);
    }
  }
}

// One phase's nine MFMA steps: the phase's weight fragments of channel blocks ob0 ..
// ob0 + OB - 1 times the samples of PB pixel rows of the sample buffer (from sbase),
// accumulated into acc; over two register buffers, step i + 1 loading while step i
// multiplies.
template <typename TC, int CPG, int PB, int OB>
__device__ __forceinline__ void dcn_phase_mfma(const DcnLayer& L, int ph, const TC* sbase, int ob0,
                                               f32x4 (&acc)[PB][OB]) {
  using Ph = DcnPhase<TC, CPG>;
  using Frag = typename Mma<TC>::Frag;
  constexpr int KG = Ph::KG, LDS_P = Ph::LDS_P;
  constexpr bool ROT = dcn_rot<TC, CPG>();
  const int lane = threadIdx.x & 63, q = lane >> 4;
  const Frag* wbase = static_cast<const Frag*>(L.wfrag) + ((size_t)ph * 9 * L.obtot + ob0) * 64 + lane;
  Frag wa0[OB], xb0[PB], wa1[OB], xb1[PB];
  auto fetch = [&](int st, Frag (&wa)[OB], Frag (&xb)[PB]) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) wa[ob] = wbase[((size_t)st * L.obtot + ob) * 64];
    // float: step st is chunk st (KG = CW = 16), quarter q its piece q
    const int so = ROT ? KG * st + 4 * dcn_piece<ROT>(st, q) : KG * st;
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) xb[pb] = Mma<TC>::ld(sbase + pb * kTW * LDS_P + so);
  };
  auto mma = [&](const Frag (&wa)[OB], const Frag (&xb)[PB]) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = Mma<TC>::step(wa[ob], xb[pb], acc[pb][ob]);
  };
  fetch(0, wa0, xb0);
#pragma unroll 1
  for (int st = 0; st < 9; st += 2) {
    if (st + 1 < 9) fetch(st + 1, wa1, xb1);
    mma(wa0, xb0);
    if (st + 1 < 9) {
      if (st + 2 < 9) fetch(st + 2, wa0, xb0);
      mma(wa1, xb1);
    }
  }
}

template <typename TF, typename TC, int C, int CPG, int PB>
__device__ __forceinline__ void dcn_tile(const DcnLayer& L, const DcnImg& im, int ty0, int tx0, TC* S) {
  using Ph = DcnPhase<TC, CPG>;
  constexpr int TH = 4 * PB;
  constexpr int OB = C / 16;
  constexpr int G = 2 * C / CPG;
  constexpr int CW = Ph::CW, GP = Ph::GP, NCH = Ph::NCH;
  constexpr int NPHASE = 2 * C / (GP * CW);
  constexpr int KG = Ph::KG;
  constexpr int QE = KG / 4;
  constexpr int NPX = TH * kTW;
  constexpr int LDS_P = Ph::LDS_P;
  static_assert(2 * C % (GP * CW) == 0 && CW % 4 == 0, "channel chunks must tile the input");

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  constexpr bool kF8 = std::is_same<TC, f8>::value;
  const TF* fa = static_cast<const TF*>(im.fa);
  const TF* fb = (im.sel != nullptr && *im.sel != 0u) ? fa : static_cast<const TF*>(im.fb);
  const float hmax = (float)im.H, wmax = (float)im.W;
  // FP8 stores samples / activation scale; folded into the bilinear-times-mask weights
  const float qs = kF8 ? *L.ainv : 1.0f;

  f32x4 acc[PB][OB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = zero4();

  constexpr bool ROT = dcn_rot<TC, CPG>();
  const TC* sbase = ROT ? &S[((wave * PB) * kTW + j) * LDS_P] : &S[((wave * PB) * kTW + j) * LDS_P + QE * q];

  // gather: item = (pixel, chunk in phase, tap), tap fastest; S[p][(gi*9 + tap)*CW + c].
  // A thread takes U items per round.  Each item always reads its four corners
  // (coordinates clamped into the map); a corner outside the map, or a pixel outside
  // the image, gets weight 0.  The rounds are software-pipelined: round r + 1's offsets
  // are loaded while round r's corner loads are in flight, and the next phase's first
  // offsets while the current phase's MFMAs run, so the two dependent global loads of
  // an item (offsets, then corners) do not both wait in every round.
  constexpr int NITEM = NPX * GP * 9;
  constexpr int U = 1;
  constexpr int NR = (NITEM + U * 256 - 1) / (U * 256);
  constexpr int NV8 = CW / 8;
  static_assert(CW % 8 == 0 || CW % 4 == 0, "chunks of 4 or 8 channels");
  struct ItemPos {
    int tap, gi, p, u, g, gy, gx;
    bool inside;
  };
  auto item_pos = [&](int item) {
    ItemPos ip;
    ip.tap = item % 9;
    const int rest = item / 9;
    ip.gi = rest % GP;
    ip.p = rest / GP;
    ip.gy = ty0 + ip.p / kTW;
    ip.gx = tx0 + (ip.p % kTW);
    ip.inside = ip.gy < im.H && ip.gx < im.W;
    return ip;
  };
  auto load_offs = [&](int ph, int r, float (&od)[U][3]) {
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int item = r * U * 256 + uu * 256 + (int)threadIdx.x;
      od[uu][0] = od[uu][1] = od[uu][2] = 0.0f;
      if (item >= NITEM) continue;
      const ItemPos ip = item_pos(item);
      const int u = ph * GP + ip.gi, g = u / NCH;
      const float* orow = im.offs + ((size_t)min(ip.gy, im.H - 1) * im.W + min(ip.gx, im.W - 1)) * L.ldo;
      od[uu][0] = orow[2 * (9 * g + ip.tap)];
      od[uu][1] = orow[2 * (9 * g + ip.tap) + 1];
      od[uu][2] = ip.inside ? orow[18 * G + 9 * g + ip.tap] : 0.0f;
    }
  };
  float od_next[U][3];
  load_offs(0, 0, od_next);

  for (int ph = 0; ph < NPHASE; ++ph) {
    if (ph) __syncthreads();
    if constexpr (CW % 8 == 0) {
      float od[2][U][3];
#pragma unroll
      for (int uu = 0; uu < U; ++uu)
#pragma unroll
        for (int k = 0; k < 3; ++k) od[0][uu][k] = od_next[uu][k];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        Raw8<TF> raw[U][4][NV8];
        float cw[U][4];
        TC* sp[U];
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
          const int item = r * U * 256 + uu * 256 + (int)threadIdx.x;
          sp[uu] = nullptr;
          if (item >= NITEM) continue;
          const ItemPos ip = item_pos(item);
          const int u = ph * GP + ip.gi;
          sp[uu] = &S[ip.p * LDS_P + (ip.gi * 9 + ip.tap) * CW];
          const int ky = ip.tap / 3, kx = ip.tap - 3 * ky;
          float m = od[r & 1][uu][2];
          if (kF8) m *= qs;
          int y0, x0;
          dcn_corners(ip.gy + ky - 1, ip.gx + kx - 1, od[r & 1][uu][0], od[r & 1][uu][1], m, im.H, im.W, y0, x0,
                      cw[uu]);
          const int ci = u * CW;
          const TF* src = ci < C ? fa : fb;
          const int cl = ci < C ? ci : ci - C;
#pragma unroll
          for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
              const int yc = min(max(y0 + cy, 0), im.H - 1), xc = min(max(x0 + cx, 0), im.W - 1);
              const TF* cp = src + ((size_t)yc * im.W + xc) * C + cl;
#pragma unroll
              for (int v = 0; v < NV8; ++v) raw[uu][2 * cy + cx][v].load(cp + 8 * v);
            }
        }
        if (r + 1 < NR) load_offs(ph, r + 1, od[(r + 1) & 1]);
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
          if (sp[uu] == nullptr) continue;
          // the chunk index within the pixel row (rotation of float 16-channel chunks)
          const int c = ROT ? (int)((sp[uu] - S) % LDS_P) / CW : 0;
          dcn_blend_store<TF, TC, NV8, ROT>(raw[uu], cw[uu], sp[uu], c);
        }
        __builtin_amdgcn_sched_barrier(0);   // keep each round's loads in their round
      }
    } else {
      // 4-channel chunks (offset groups of fewer than 8 channels): one item at a time
      for (int item = (int)threadIdx.x; item < NITEM; item += 256) {
        const ItemPos ip = item_pos(item);
        const int u = ph * GP + ip.gi, g = u / NCH;
        TC* sp = &S[ip.p * LDS_P + (ip.gi * 9 + ip.tap) * CW];
        const int ky = ip.tap / 3, kx = ip.tap - 3 * ky;
        const float* orow = im.offs + ((size_t)min(ip.gy, im.H - 1) * im.W + min(ip.gx, im.W - 1)) * L.ldo;
        float m = ip.inside ? orow[18 * G + 9 * g + ip.tap] : 0.0f;
        if (kF8) m *= qs;
        const float py = fminf(fmaxf((float)(ip.gy + ky - 1) + orow[2 * (9 * g + ip.tap)], -2.0f), hmax + 1.0f);
        const float px = fminf(fmaxf((float)(ip.gx + kx - 1) + orow[2 * (9 * g + ip.tap) + 1], -2.0f), wmax + 1.0f);
        const float y0f = floorf(py), x0f = floorf(px);
        const float ly = py - y0f, lx = px - x0f;
        const int y0 = (int)y0f, x0 = (int)x0f;
        const int ci = u * CW;
        const TF* src = ci < C ? fa : fb;
        const int cl = ci < C ? ci : ci - C;
        float cw[4];
        const TF* cp[4];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const int yy = y0 + cy, xx = x0 + cx;
            const bool ok = yy >= 0 && yy < im.H && xx >= 0 && xx < im.W;
            const int yc = min(max(yy, 0), im.H - 1), xc = min(max(xx, 0), im.W - 1);
            cw[2 * cy + cx] = ok ? (cy ? ly : 1.0f - ly) * (cx ? lx : 1.0f - lx) * m : 0.0f;
            cp[2 * cy + cx] = src + ((size_t)yc * im.W + xc) * C + cl;
          }
#pragma unroll
        for (int v = 0; v < CW; v += 4) {
          f32x4 acc4 = zero4();
#pragma unroll
          for (int k = 0; k < 4; ++k) acc4 += cw[k] * load4f<TF>(cp[k] + v);
          store4f<TC>(sp + v, acc4);
        }
      }
    }
    __syncthreads();
    if (ph + 1 < NPHASE) load_offs(ph + 1, 0, od_next);
    dcn_phase_mfma<TC, CPG, PB, OB>(L, ph, sbase, 0, acc);
  }

  dcn_store<TF, TC, C, PB, DcnSmem<TC, CPG, PB>::N>(L, im, ty0, tx0, acc, S);
}

template <typename TF, typename TC, int C, int CPG, int PB>
__global__ __launch_bounds__(256) void k_dcn(DcnLayer L, DcnImg im) {
  __shared__ __attribute__((aligned(16))) TC S[DcnSmem<TC, CPG, PB>::N];
  const int tiles_x = (im.W + kTW - 1) / kTW;
  const int ntile = tiles_x * ((im.H + 4 * PB - 1) / (4 * PB));
  const int t = xcd_tile(blockIdx.x, ntile);
  dcn_tile<TF, TC, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, S);
}

template <typename TF, typename TC, int C, int CPG, int PB>
__global__ __launch_bounds__(256) void k_dcn_batch(DcnLayer L, const DcnImg* __restrict__ jobs,
                                                   const int* __restrict__ count) {
  __shared__ __attribute__((aligned(16))) TC S[DcnSmem<TC, CPG, PB>::N];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const DcnImg im = jobs[find_job(jobs, njobs, item)];
    const int t = item - im.item_begin;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    dcn_tile<TF, TC, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, S);
    __syncthreads();
  }
}

// ---- windowed DCN: a phase's corners read from an LDS copy of the sampled window ----
// Same phases, steps and reduction order as dcn_tile, and every sample formed with the
// same arithmetic (corner weights, four fused multiply-adds in corner order, one
// rounding to the MFMA type), so the output is bit-identical; what changes is where the
// corners are read and that no sample buffer is written.  A phase covers KG channels of
// one map.  Per phase: the offsets and masks of its groups for the tile's pixels are
// copied to LDS by coalesced loads, and the threads that load them also reduce the
// bounding box of the sampling positions; when the box fits FH x FW pixels, that window
// of the map is copied to LDS (pixels outside the map as zeros: their corner weights
// are zero) and the corners are read there, otherwise from the map itself.  Each lane
// forms the B operand of every MFMA step in registers from one item (its fragment's E
// channels lie in one chunk) per pixel row.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

template <typename T, int C, int CPG, int PB>
struct DcnWin {
  static constexpr int KG = Mma<T>::KG;
  static constexpr int E = 16 / (int)sizeof(T);       // channels of one 16-byte fragment
  static constexpr int CW = CPG < KG ? CPG : KG;
  static constexpr int TH = 4 * PB;
  static constexpr int FH = TH + 8, FW = 24;           // window: sample spread up to about 5 pixels
  static constexpr int WP = KG;                        // window pixel stride (elements): 64 bytes
  // offset groups of a phase and the floats of a pixel's staged offsets and masks
  static constexpr int NG = KG / CW >= CPG / CW ? (KG / CW) / (CPG / CW) : 1;
  static constexpr int OPS = (27 * NG + 1) & ~1;
  static constexpr int NWIN = FH * FW * WP;            // window elements (T)
  static constexpr int NOFF = TH * kTW * OPS;          // staged offsets (float), after the window
  static constexpr int BYTES = NWIN * (int)sizeof(T) + NOFF * 4;
  static constexpr int OLDP = C + E;                   // output staging row (as in dcn_tile)
  static_assert(CW % E == 0, "a fragment's channels lie in one chunk");
  static_assert(NWIN * (int)sizeof(T) % 16 == 0, "the offsets start 16-byte aligned");
  static_assert(TH * kTW * OLDP * (int)sizeof(T) <= BYTES, "the output tile fits the buffer");
};

// The E channels at p as floats (16-bit types: lo and hi; float: lo).
template <typename T>
__device__ __forceinline__ void frag_f32(u32x4 r, f32x4& lo, f32x4& hi) {
  Raw8<T> w;
  w.v = r;
  w.to_f32(lo, hi);
}
template <>
__device__ __forceinline__ void frag_f32<float>(u32x4 r, f32x4& lo, f32x4& hi) {
  lo = __builtin_bit_cast(f32x4, r);
  hi = zero4();
}
// The fragment in the MFMA type, rounded as dcn_tile's sample buffer stores it.
template <typename T>
__device__ __forceinline__ u32x4 frag_pack(f32x4 lo, f32x4 hi) {
  typedef T T8 __attribute__((ext_vector_type(8)));
  const T8 v = T8{(T)lo[0], (T)lo[1], (T)lo[2], (T)lo[3], (T)hi[0], (T)hi[1], (T)hi[2], (T)hi[3]};
  return __builtin_bit_cast(u32x4, v);
}
template <>
__device__ __forceinline__ u32x4 frag_pack<float>(f32x4 lo, f32x4) {
  return __builtin_bit_cast(u32x4, lo);
}

template <typename T, int C, int CPG, int PB>
__device__ __forceinline__ void dcnw_tile(const DcnLayer& L, const DcnImg& im, int ty0, int tx0, uint8_t* smem,
                                          int (*red)[16]) {
  using D = DcnWin<T, C, CPG, PB>;
  constexpr int KG = D::KG, E = D::E, CW = D::CW, FH = D::FH, FW = D::FW, WP = D::WP, TH = D::TH;
  constexpr int GP = KG / CW, NCH = CPG / CW;
  constexpr int G = 2 * C / CPG;
  constexpr int NPHASE = 2 * C / KG;
  constexpr int OB = C / 16;
  constexpr int NG = D::NG, OPS = D::OPS;
  constexpr int NOL = TH * kTW * 18 * NG;              // loads: 9 NG pairs and 9 NG masks per pixel
  constexpr bool SIXTEEN = sizeof(T) == 2;
  static_assert(C % KG == 0, "a phase's channels lie in one map");
  using Frag = typename Mma<T>::Frag;

  T* Wn = reinterpret_cast<T*>(smem);
  float* Of = reinterpret_cast<float*>(smem + D::NWIN * sizeof(T));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const T* fa = static_cast<const T*>(im.fa);
  const T* fb = (im.sel != nullptr && *im.sel != 0u) ? fa : static_cast<const T*>(im.fb);
  const float hmax = (float)im.H, wmax = (float)im.W;
  const int gx = tx0 + j;

  f32x4 acc[PB][OB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = zero4();

  for (int ph = 0; ph < NPHASE; ++ph) {
    const int g0 = ph * GP / NCH;
    // after the previous phase's reads of the window and the offsets
    if (ph) __syncthreads();
    // the phase's offsets and masks for the tile's pixels: per pixel OPS floats, the
    // (dy, dx) of group g0 + gl, tap t at 2 (9 gl + t), the masks after them at
    // 18 NG + 9 gl + t; the loaders of the (dy, dx) pairs reduce the corner box
    int ylo = 1 << 30, yhi = -(1 << 30), xlo = 1 << 30, xhi = -(1 << 30);
#pragma unroll 6
    for (int idx = (int)threadIdx.x; idx < NOL; idx += 256) {
      const int p = idx / (18 * NG), k = idx - p * (18 * NG);
      const int py0 = ty0 + p / kTW, px0 = tx0 + p % kTW;
      const float* orow = im.offs + ((size_t)min(py0, im.H - 1) * im.W + min(px0, im.W - 1)) * L.ldo;
      if (k < 9 * NG) {
        const f32x2 d = *reinterpret_cast<const f32x2*>(orow + 18 * g0 + 2 * k);
        *reinterpret_cast<f32x2*>(&Of[p * OPS + 2 * k]) = d;
        const int tap = k % 9, ky = tap / 3, kx = tap - 3 * ky;
        // the positions exactly as the steps below form them
        const float py = fminf(fmaxf((float)(py0 + ky - 1) + d[0], -2.0f), hmax + 1.0f);
        const float px = fminf(fmaxf((float)(px0 + kx - 1) + d[1], -2.0f), wmax + 1.0f);
        const int y0 = (int)floorf(py), x0 = (int)floorf(px);
        ylo = min(ylo, y0);
        yhi = max(yhi, y0);
        xlo = min(xlo, x0);
        xhi = max(xhi, x0);
      } else {
        const int m = k - 9 * NG;
        Of[p * OPS + 18 * NG + m] = orow[18 * G + 9 * g0 + m];
      }
    }
    ylo = wave_min(ylo);
    yhi = wave_max(yhi);
    xlo = wave_min(xlo);
    xhi = wave_max(xhi);
    int* rd = red[ph & 1];
    if (lane == 0) {
      rd[4 * wave] = ylo;
      rd[4 * wave + 1] = yhi;
      rd[4 * wave + 2] = xlo;
      rd[4 * wave + 3] = xhi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      ylo = min(ylo, rd[4 * w]);
      yhi = max(yhi, rd[4 * w + 1]);
      xlo = min(xlo, rd[4 * w + 2]);
      xhi = max(xhi, rd[4 * w + 3]);
    }
    const int wy0 = ylo, wx0 = xlo, nh = yhi - ylo + 2, nw = xhi - xlo + 2;
    const bool win = nh <= FH && nw <= FW;
    const T* map = ph * KG < C ? fa : fb;
    const int cl0 = (ph * KG) % C;
    if (win) {
      constexpr int PPX = KG / E;                     // 16-byte pieces of a window pixel
      constexpr int NPC = FH * FW * PPX;
      constexpr int NIT = (NPC + 255) / 256, BAT = 4;
      // in batches of BAT loads per thread (all in flight, then stored)
#pragma unroll 1
      for (int k0 = 0; k0 < NIT; k0 += BAT) {
        u32x4 v[BAT];
#pragma unroll
        for (int k = 0; k < BAT; ++k) {
          const int idx = (int)threadIdx.x + 256 * (k0 + k);
          const int p = idx / PPX, pc = idx - p * PPX;
          const int r = p / FW, c = p - r * FW;
          const int yy = wy0 + r, xx = wx0 + c;
          v[k] = u32x4{0u, 0u, 0u, 0u};
          if (idx < NPC && r < nh && c < nw && yy >= 0 && yy < im.H && xx >= 0 && xx < im.W)
            v[k] = ldu4(map + ((size_t)yy * im.W + xx) * C + cl0 + E * pc);
        }
#pragma unroll
        for (int k = 0; k < BAT; ++k) {
          const int idx = (int)threadIdx.x + 256 * (k0 + k);
          const int p = idx / PPX, pc = idx - p * PPX;
          const int r = p / FW, c = p - r * FW;
          if (idx < NPC && r < nh && c < nw) stu4(&Wn[p * WP + E * pc], v[k]);
        }
      }
    }
    // the staged offsets (and the window) visible to every lane
    __syncthreads();

    const Frag* wbase = static_cast<const Frag*>(L.wfrag) + ((size_t)ph * 9 * L.obtot) * 64 + lane;
    auto steps = [&](auto in_window) {
      constexpr bool WIN = decltype(in_window)::value;
      Frag wa[OB];
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) wa[ob] = wbase[(size_t)ob * 64];
#pragma unroll 1
      for (int st = 0; st < 9; ++st) {
        // the lane's item: K index st KG + E q of the phase, in chunk-major order
        const int k0 = st * KG + E * q;
        const int it = k0 / CW, gi = it / 9, tap = it - 9 * gi;
        const int gl = (ph * GP + gi) / NCH - g0;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int wch = gi * CW + k0 % CW;           // channel within the phase's KG
        Frag wn[OB];
        if (st + 1 < 9) {
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) wn[ob] = wbase[((size_t)(st + 1) * L.obtot + ob) * 64];
        }
        Frag xb[PB];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          const int gy = ty0 + wave * PB + pb;
          const float* o = &Of[((wave * PB + pb) * kTW + j) * OPS];
          const f32x2 d = *reinterpret_cast<const f32x2*>(&o[2 * (9 * gl + tap)]);
          const float m = (gy < im.H && gx < im.W) ? o[18 * NG + 9 * gl + tap] : 0.0f;
          // beyond one pixel outside the map every sample is zero; the clamp keeps the
          // integer conversion defined for any offset value
          const float py = fminf(fmaxf((float)(gy + ky - 1) + d[0], -2.0f), hmax + 1.0f);
          const float px = fminf(fmaxf((float)(gx + kx - 1) + d[1], -2.0f), wmax + 1.0f);
          const float y0f = floorf(py), x0f = floorf(px);
          const float ly = py - y0f, lx = px - x0f;
          const int y0 = (int)y0f, x0 = (int)x0f;
          u32x4 raw[4];
          float cw[4];
#pragma unroll
          for (int cy = 0; cy < 2; ++cy)
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
              const int yy = y0 + cy, xx = x0 + cx;
              const bool ok = yy >= 0 && yy < im.H && xx >= 0 && xx < im.W;
              cw[2 * cy + cx] = ok ? (cy ? ly : 1.0f - ly) * (cx ? lx : 1.0f - lx) * m : 0.0f;
              if constexpr (WIN) {
                raw[2 * cy + cx] = ldu4(&Wn[((yy - wy0) * FW + (xx - wx0)) * WP + wch]);
              } else {
                const int yc = min(max(yy, 0), im.H - 1), xc = min(max(xx, 0), im.W - 1);
                raw[2 * cy + cx] = ldu4(map + ((size_t)yc * im.W + xc) * C + cl0 + wch);
              }
            }
          f32x4 lo = zero4(), hi = zero4();
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            f32x4 a, b;
            frag_f32<T>(raw[k], a, b);
            lo += cw[k] * a;
            if constexpr (SIXTEEN) hi += cw[k] * b;
          }
          xb[pb] = frag_pack<T>(lo, hi);
        }
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = Mma<T>::step(wa[ob], xb[pb], acc[pb][ob]);
        if (st + 1 < 9) {
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) wa[ob] = wn[ob];
        }
      }
    };
    if (win) steps(std::true_type{});
    else steps(std::false_type{});
  }
  dcn_store<T, T, C, PB, D::BYTES / (int)sizeof(T)>(L, im, ty0, tx0, acc, reinterpret_cast<T*>(smem));
}

// Three workgroups per CU where their LDS fits three times, else two.
template <typename T, int C, int CPG, int PB>
constexpr int dcnw_waves() {
  return 3 * (DcnWin<T, C, CPG, PB>::BYTES + 128) <= 163840 ? 3 : 2;
}

template <typename T, int C, int CPG, int PB>
__global__ __launch_bounds__(256, (dcnw_waves<T, C, CPG, PB>())) void k_dcnw(DcnLayer L, DcnImg im) {
  __shared__ __attribute__((aligned(16))) uint8_t Wn[DcnWin<T, C, CPG, PB>::BYTES];
  __shared__ int red[2][16];
  const int tiles_x = (im.W + kTW - 1) / kTW;
  const int ntile = tiles_x * ((im.H + 4 * PB - 1) / (4 * PB));
  const int t = xcd_tile(blockIdx.x, ntile);
  dcnw_tile<T, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, Wn, red);
}

template <typename T, int C, int CPG, int PB>
__global__ __launch_bounds__(256, (dcnw_waves<T, C, CPG, PB>())) void k_dcnw_batch(DcnLayer L,
                                                                                  const DcnImg* __restrict__ jobs,
                                                                                  const int* __restrict__ count) {
  __shared__ __attribute__((aligned(16))) uint8_t Wn[DcnWin<T, C, CPG, PB>::BYTES];
  __shared__ int red[2][16];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const DcnImg im = jobs[find_job(jobs, njobs, item)];
    const int t = item - im.item_begin;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    dcnw_tile<T, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, Wn, red);
    __syncthreads();
  }
}

// ---- staged form: the plain form's items and sample buffer, corners from LDS ----
// Per phase the plain form's gather items (pixel, chunk, tap) first load their offsets and
// form their sampling positions; the workgroup reduces the box of all their corners and,
// when it fits FH x FW pixels, copies the phase's KG channels of that box from the map
// into LDS with whole-pixel loads (coordinates clamped into the map, as the plain form
// clamps its corner reads).  The items then read their four corners from that copy
// instead of from global memory, blend them into the same sample buffer with the same
// arithmetic, and the same MFMA steps follow: the output is bit-identical to the plain
// form's.  A phase whose box does not fit reads its corners from the maps.
template <typename T, int C, int CPG, int PB>
struct DcnStaged {
  static constexpr int KG = Mma<T>::KG;
  static constexpr int TH = 4 * PB;
  static constexpr int FH = TH + 7, FW = kTW + 6;      // samples within about 2.5 pixels of the tile
  static constexpr int WP = KG;                        // window pixel stride (elements): 64 bytes
  // window row stride: 16 bytes of padding, so that the nine taps of an item (three
  // rows, three columns) fall in different LDS bank groups
  static constexpr int WR = FW * WP + 16 / (int)sizeof(T);
  static constexpr int NS = DcnSmem<T, CPG, PB>::N;    // the sample buffer (elements)
  static constexpr int NWIN = FH * WR;
  static constexpr int BYTES = (NS + NWIN) * (int)sizeof(T);
  static_assert(NS * (int)sizeof(T) % 16 == 0, "the window starts 16-byte aligned");
};

template <typename T, int C, int CPG, int PB>
__device__ __forceinline__ void dcns_tile(const DcnLayer& L, const DcnImg& im, int ty0, int tx0, T* S, T* Wn,
                                          int* red) {
  using Ph = DcnPhase<T, CPG>;
  using D = DcnStaged<T, C, CPG, PB>;
  constexpr int TH = 4 * PB, OB = C / 16, G = 2 * C / CPG;
  constexpr int CW = Ph::CW, GP = Ph::GP, NCH = Ph::NCH, KG = Ph::KG, QE = KG / 4, LDS_P = Ph::LDS_P;
  constexpr int NPHASE = 2 * C / KG;
  constexpr int NPX = TH * kTW, NITEM = NPX * GP * 9, NR = (NITEM + 255) / 256, NV8 = CW / 8;
  constexpr int FH = D::FH, FW = D::FW, WP = D::WP, WR = D::WR;
  constexpr int E = 16 / (int)sizeof(T), PPX = KG / E;
  constexpr bool ROT = dcn_rot<T, CPG>();
  static_assert(CW % 8 == 0 && C % KG == 0, "chunks of whole 8-channel vectors; a phase in one map");

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const T* fa = static_cast<const T*>(im.fa);
  const T* fb = (im.sel != nullptr && *im.sel != 0u) ? fa : static_cast<const T*>(im.fb);

  // 64 channels: each wave multiplies one block of 16 output channels over all TH rows
  // (a quarter of the phase's weight fragments per wave), else PB rows over all blocks
  constexpr bool CS = OB == 4;
  constexpr int AR = CS ? TH : PB, AB = CS ? 1 : OB;
  f32x4 acc[AR][AB];
#pragma unroll
  for (int r = 0; r < AR; ++r)
#pragma unroll
    for (int b = 0; b < AB; ++b) acc[r][b] = zero4();
  const int r0 = CS ? 0 : wave * PB;
  const T* sbase = ROT ? &S[(r0 * kTW + j) * LDS_P] : &S[(r0 * kTW + j) * LDS_P + QE * q];

  // item r of this thread: (pixel, chunk gi, tap) as in the plain form, tap fastest
  auto item_of = [&](int r, int& tap, int& gi, int& p) {
    const int item = r * 256 + (int)threadIdx.x;
    tap = item % 9;
    const int rest = item / 9;
    gi = rest % GP;
    p = rest / GP;
    return (r + 1) * 256 <= NITEM || item < NITEM;   // rounds below NITEM / 256 are full
  };
  // offsets (dy, dx) and mask of every item of phase ph, all rounds in flight at once
  float od[NR][3];
  auto load_offs = [&](int ph) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      int tap, gi, p;
      od[r][0] = od[r][1] = od[r][2] = 0.0f;
      if (!item_of(r, tap, gi, p)) continue;
      const int g = (ph * GP + gi) / NCH;
      const int gy = ty0 + p / kTW, gx = tx0 + p % kTW;
      const float* orow = im.offs + ((size_t)min(gy, im.H - 1) * im.W + min(gx, im.W - 1)) * L.ldo;
      od[r][0] = orow[2 * (9 * g + tap)];
      od[r][1] = orow[2 * (9 * g + tap) + 1];
      od[r][2] = gy < im.H && gx < im.W ? orow[18 * G + 9 * g + tap] : 0.0f;
    }
  };
  load_offs(0);

  for (int ph = 0; ph < NPHASE; ++ph) {
    // the box of the phase's corners (rows y0 .. y0 + 1, columns x0 .. x0 + 1 of every item)
    int ylo = 1 << 30, yhi = -(1 << 30), xlo = 1 << 30, xhi = -(1 << 30);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      int tap, gi, p;
      if (!item_of(r, tap, gi, p)) continue;
      const int ky = tap / 3, kx = tap - 3 * ky;
      int y0, x0;
      float cw[4];
      dcn_corners(ty0 + p / kTW + ky - 1, tx0 + p % kTW + kx - 1, od[r][0], od[r][1], od[r][2], im.H, im.W, y0,
                  x0, cw);
      ylo = min(ylo, y0);
      yhi = max(yhi, y0);
      xlo = min(xlo, x0);
      xhi = max(xhi, x0);
    }
    ylo = wave_min(ylo);
    yhi = wave_max(yhi);
    xlo = wave_min(xlo);
    xhi = wave_max(xhi);
    if (lane == 0) {
      red[4 * wave] = ylo;
      red[4 * wave + 1] = yhi;
      red[4 * wave + 2] = xlo;
      red[4 * wave + 3] = xhi;
    }
    // also: the previous phase's MFMA reads of the sample buffer are done
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      ylo = min(ylo, red[4 * w]);
      yhi = max(yhi, red[4 * w + 1]);
      xlo = min(xlo, red[4 * w + 2]);
      xhi = max(xhi, red[4 * w + 3]);
    }
    const int wy0 = ylo, wx0 = xlo, nh = yhi - ylo + 2, nw = xhi - xlo + 2;
    const bool win = nh <= FH && nw <= FW;
    const T* map = ph * KG < C ? fa : fb;
    const int cl0 = (ph * KG) % C;
    if (win) {
      constexpr int NPC = FH * FW * PPX, NIT = (NPC + 255) / 256;
      u32x4 v[NIT];
#pragma unroll
      for (int k = 0; k < NIT; ++k) {
        const int idx = (int)threadIdx.x + 256 * k;
        const int px = idx / PPX, pc = idx - px * PPX;
        const int r = px / FW, c = px - r * FW;
        v[k] = u32x4{0u, 0u, 0u, 0u};
        if (idx < NPC && r < nh && c < nw) {
          const int yy = min(max(wy0 + r, 0), im.H - 1), xx = min(max(wx0 + c, 0), im.W - 1);
          v[k] = ldu4(map + ((size_t)yy * im.W + xx) * C + cl0 + E * pc);
        }
      }
#pragma unroll
      for (int k = 0; k < NIT; ++k) {
        const int idx = (int)threadIdx.x + 256 * k;
        const int px = idx / PPX, pc = idx - px * PPX;
        const int r = px / FW, c = px - r * FW;
        if (idx < NPC && r < nh && c < nw) stu4(&Wn[r * WR + c * WP + E * pc], v[k]);
      }
      // the window visible to every lane
      __syncthreads();
    }
    // gather: the items' corners from the window (or the map), blended into S; one loop
    // per source, so that the window reads are LDS reads
    auto gather = [&](auto in_window) {
      constexpr bool WIN = decltype(in_window)::value;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        int tap, gi, p;
        if (!item_of(r, tap, gi, p)) continue;
        const int ky = tap / 3, kx = tap - 3 * ky;
        int y0, x0;
        float cw[4];
        dcn_corners(ty0 + p / kTW + ky - 1, tx0 + p % kTW + kx - 1, od[r][0], od[r][1], od[r][2], im.H, im.W, y0,
                    x0, cw);
        Raw8<T> raw[4][NV8];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            if constexpr (WIN) {
              const T* cp = &Wn[(y0 + cy - wy0) * WR + (x0 + cx - wx0) * WP + gi * CW];
#pragma unroll
              for (int v8 = 0; v8 < NV8; ++v8) raw[2 * cy + cx][v8].load(cp + 8 * v8);
            } else {
              const int yc = min(max(y0 + cy, 0), im.H - 1), xc = min(max(x0 + cx, 0), im.W - 1);
              const T* cp = map + ((size_t)yc * im.W + xc) * C + cl0 + gi * CW;
#pragma unroll
              for (int v8 = 0; v8 < NV8; ++v8) raw[2 * cy + cx][v8].load(cp + 8 * v8);
            }
          }
        const int chunk = gi * 9 + tap;   // the chunk index within the pixel row
        dcn_blend_store<T, T, NV8, ROT>(raw, cw, &S[p * LDS_P + chunk * CW], chunk);
      }
    };
    if (win) gather(std::true_type{});
    else gather(std::false_type{});
    // the samples visible to every wave
    __syncthreads();
    if (ph + 1 < NPHASE) load_offs(ph + 1);
    dcn_phase_mfma<T, CPG, AR, AB>(L, ph, sbase, CS ? wave : 0, acc);
  }
  dcn_store<T, T, C, AR, D::NS, CS, AB>(L, im, ty0, tx0, acc, S);
}

// Three workgroups per CU where the registers allow it (up to five gather rounds of at
// most 32 bytes per corner), else two.
template <typename T, int C, int CPG, int PB>
constexpr int dcns_waves() {
  using Ph = DcnPhase<T, CPG>;
  return 4 * PB * kTW * Ph::GP * 9 <= 5 * 256 && Ph::CW * (int)sizeof(T) <= 64 ? 3 : 2;
}

template <typename T, int C, int CPG, int PB>
__global__ __launch_bounds__(256, (dcns_waves<T, C, CPG, PB>())) void k_dcns(DcnLayer L, DcnImg im) {
  using D = DcnStaged<T, C, CPG, PB>;
  __shared__ __attribute__((aligned(16))) T S[D::NS + D::NWIN];
  __shared__ int red[16];
  const int tiles_x = (im.W + kTW - 1) / kTW;
  const int ntile = tiles_x * ((im.H + 4 * PB - 1) / (4 * PB));
  const int t = xcd_tile(blockIdx.x, ntile);
  dcns_tile<T, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, S, S + D::NS, red);
}

template <typename T, int C, int CPG, int PB>
__global__ __launch_bounds__(256, (dcns_waves<T, C, CPG, PB>())) void k_dcns_batch(DcnLayer L,
                                                                                  const DcnImg* __restrict__ jobs,
                                                                                  const int* __restrict__ count) {
  using D = DcnStaged<T, C, CPG, PB>;
  __shared__ __attribute__((aligned(16))) T S[D::NS + D::NWIN];
  __shared__ int red[16];
  const int njobs = count[0], total = count[1];
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const DcnImg im = jobs[find_job(jobs, njobs, item)];
    const int t = item - im.item_begin;
    const int tiles_x = (im.W + kTW - 1) / kTW;
    dcns_tile<T, C, CPG, PB>(L, im, (t / tiles_x) * 4 * PB, (t % tiles_x) * kTW, S, S + D::NS, red);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- dispatch ----

template <typename TF, typename TC, int C, int CPG, int PB>
void run_dcn(const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count, hipStream_t s) {
  if (im) {
    const int ntile = ((im->W + kTW - 1) / kTW) * ((im->H + 4 * PB - 1) / (4 * PB));
    hipLaunchKernelGGL((k_dcn<TF, TC, C, CPG, PB>), dim3(ntile), dim3(256), 0, s, L, *im);
  } else {
    hipLaunchKernelGGL((k_dcn_batch<TF, TC, C, CPG, PB>), dim3(kBatchGrid), dim3(256), 0, s, L, jobs, count);
  }
}

template <typename T, int C, int CPG, int PB>
void run_dcnw(const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count, hipStream_t s) {
  if (im) {
    const int ntile = ((im->W + kTW - 1) / kTW) * ((im->H + 4 * PB - 1) / (4 * PB));
    hipLaunchKernelGGL((k_dcnw<T, C, CPG, PB>), dim3(ntile), dim3(256), 0, s, L, *im);
  } else {
    hipLaunchKernelGGL((k_dcnw_batch<T, C, CPG, PB>), dim3(kBatchGrid), dim3(256), 0, s, L, jobs, count);
  }
}

template <typename T, int C, int CPG, int PB>
void run_dcns(const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count, hipStream_t s) {
  if (im) {
    const int ntile = ((im->W + kTW - 1) / kTW) * ((im->H + 4 * PB - 1) / (4 * PB));
    hipLaunchKernelGGL((k_dcns<T, C, CPG, PB>), dim3(ntile), dim3(256), 0, s, L, *im);
  } else {
    hipLaunchKernelGGL((k_dcns_batch<T, C, CPG, PB>), dim3(kBatchGrid), dim3(256), 0, s, L, jobs, count);
  }
}

// Staged form: float and 16-bit maps with chunks of 8 or more channels (8 or more
// channels per offset group).
template <typename T, int PB>
hipError_t dcns_c(int C, int cpg, const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count,
                  hipStream_t s) {
  if (C == 64) {
    switch (cpg) {
      case 8: run_dcns<T, 64, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcns<T, 64, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcns<T, 64, 32, PB>(L, im, jobs, count, s); break;
      case 64: run_dcns<T, 64, 64, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else if (C == 32) {
    switch (cpg) {
      case 8: run_dcns<T, 32, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcns<T, 32, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcns<T, 32, 32, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Windowed form: float and 16-bit maps whose chunks hold at least one fragment's
// channels (16-bit: 8 or more channels per offset group).
template <typename T, int PB>
hipError_t dcnw_c(int C, int cpg, const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count,
                  hipStream_t s) {
  constexpr bool F32 = std::is_same<T, float>::value;
  if (C == 64) {
    switch (cpg) {
      case 4:
        if constexpr (F32) { run_dcnw<T, 64, 4, PB>(L, im, jobs, count, s); break; }
        return hipErrorInvalidValue;
      case 8: run_dcnw<T, 64, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcnw<T, 64, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcnw<T, 64, 32, PB>(L, im, jobs, count, s); break;
      case 64: run_dcnw<T, 64, 64, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else if (C == 32) {
    switch (cpg) {
      case 4:
        if constexpr (F32) { run_dcnw<T, 32, 4, PB>(L, im, jobs, count, s); break; }
        return hipErrorInvalidValue;
      case 8: run_dcnw<T, 32, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcnw<T, 32, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcnw<T, 32, 32, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// FP8: float16 storage, e4m3 samples and weights, 64 channels; one pixel row per wave
// (a phase holds all 2C channels x 9 taps of a tile in LDS).
hipError_t dcn_f8(int cpg, const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count,
                  hipStream_t s) {
  switch (cpg) {
    case 4: run_dcn<f16, f8, 64, 4, 1>(L, im, jobs, count, s); break;
    case 8: run_dcn<f16, f8, 64, 8, 1>(L, im, jobs, count, s); break;
    case 16: run_dcn<f16, f8, 64, 16, 1>(L, im, jobs, count, s); break;
    case 32: run_dcn<f16, f8, 64, 32, 1>(L, im, jobs, count, s); break;
    case 64: run_dcn<f16, f8, 64, 64, 1>(L, im, jobs, count, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TF, int PB>
hipError_t dcn_c(int C, int cpg, const DcnLayer& L, const DcnImg* im, const DcnImg* jobs, const int* count,
                 hipStream_t s) {
  // cpg = 2C / offset groups: 4 .. 2C
  if (C == 64) {
    switch (cpg) {
      case 4: run_dcn<TF, TF, 64, 4, PB>(L, im, jobs, count, s); break;
      case 8: run_dcn<TF, TF, 64, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcn<TF, TF, 64, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcn<TF, TF, 64, 32, PB>(L, im, jobs, count, s); break;
      case 64: run_dcn<TF, TF, 64, 64, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else if (C == 32) {
    switch (cpg) {
      case 4: run_dcn<TF, TF, 32, 4, PB>(L, im, jobs, count, s); break;
      case 8: run_dcn<TF, TF, 32, 8, PB>(L, im, jobs, count, s); break;
      case 16: run_dcn<TF, TF, 32, 16, PB>(L, im, jobs, count, s); break;
      case 32: run_dcn<TF, TF, 32, 32, PB>(L, im, jobs, count, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TF>
hipError_t dcn_pb(int pb, int C, int cpg, const DcnLayer& L, const DcnImg* im, const DcnImg* jobs,
                  const int* count, hipStream_t s) {
  if (pb == 1) return dcn_c<TF, 1>(C, cpg, L, im, jobs, count, s);
  if (pb == 2) return dcn_c<TF, 2>(C, cpg, L, im, jobs, count, s);
  if (pb == (1 | kDcnWindow)) return dcnw_c<TF, 1>(C, cpg, L, im, jobs, count, s);
  if (pb == (2 | kDcnWindow)) return dcnw_c<TF, 2>(C, cpg, L, im, jobs, count, s);
  if (pb == (1 | kDcnStaged)) return dcns_c<TF, 1>(C, cpg, L, im, jobs, count, s);
  return hipErrorInvalidValue;
}

hipError_t dcn_dispatch(const PackedConv& P, int tf, int pb, int ldo, int groups, const DcnImg* im,
                        const DcnImg* jobs, const int* count, hipStream_t s) {
  DcnLayer L;
  L.wfrag = P.frag;
  L.bias = P.bias;
  L.oscale = P.oscale;
  L.ainv = P.ainv;
  L.ldo = ldo;
  L.groups = groups;
  L.obtot = P.obtot;
  const int cpg = 2 * P.cout / groups;
  if (P.tc == DT_F8) {
    if (tf != DT_F16 || P.cout != 64 || pb != 1 || !P.oscale || !P.ainv) return hipErrorInvalidValue;
    return dcn_f8(cpg, L, im, jobs, count, s);
  }
  if (P.tc != tf) return hipErrorInvalidValue;
  switch (tf) {
    case DT_F32: return dcn_pb<float>(pb, P.cout, cpg, L, im, jobs, count, s);
    case DT_F16: return dcn_pb<f16>(pb, P.cout, cpg, L, im, jobs, count, s);
    case DT_BF16: return dcn_pb<bf16>(pb, P.cout, cpg, L, im, jobs, count, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_dcn(const PackedConv& P, int tf, int pb, const DcnImg& im, int ldo, int groups,
                      hipStream_t s) {
  return dcn_dispatch(P, tf, pb, ldo, groups, &im, nullptr, nullptr, s);
}

hipError_t launch_dcn_batch(const PackedConv& P, int tf, int pb, const DcnImg* jobs, const int* count,
                            int ldo, int groups, hipStream_t s) {
  return dcn_dispatch(P, tf, pb, ldo, groups, nullptr, jobs, count, s);
}

}  // namespace nv

// Network kernels (gfx950): 3x3 convolutions as implicit GEMM on MFMA, the modulated
// deformable convolution with its bilinear gather fused into the B-operand load, and
// the two thin convolutions (3 -> C in, C -> 3 out) on the vector ALUs.
//
// Activations are NHWC float32.  A workgroup owns a tile of TH x 16 output pixels
// (TH = 4 waves x PB rows) and OB blocks of 16 output channels.  In the MFMA the
// weights are the A operand (rows = output channels) and the activations the B
// operand (columns = the 16 pixels of one tile row), so each lane ends up holding four
// consecutive output channels of one pixel: one 16-byte store per accumulator.
//
// The reduction index K = (tap, input channel) is consumed in groups of 16 channels;
// within a group, lane quarter q takes channels 4q..4q+3 over the four k-steps, so the
// B operand of four MFMAs is one 16-byte LDS read and the A operand one 16-byte global
// read (weights are pre-arranged in exactly that fragment order).
#include "nv_device.h"
#include "nv_internal.h"

namespace nv {
namespace {

constexpr int kTW = 16;

struct ConvArgs {
  const float* src0;
  const float* src1;
  const uint32_t* sel;   // when non-null and *sel != 0, alt0/alt1 (if set) replace src0/src1
  const float* alt0;
  const float* alt1;
  const f32x4* wfrag;
  const float* bias;
  const float* res;
  float* dst;
  int H, W;
  int ldy;      // channel stride of dst / res
  int cout;     // real output channels (EPI_OFFSET stores only these)
  int sig_lo;   // EPI_OFFSET: sigmoid on channels >= sig_lo
  int obtot;    // total 16-channel output blocks of the layer
  int ccout;    // EPI_SHUFFLE: channels of the high-resolution map
};

template <int CCH, int NCHUNK, int OB, int PB, int EPI>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a) {
  constexpr int TH = 4 * PB;
  constexpr int LDP = CCH + 4;                 // padded pixel stride in LDS (floats)
  constexpr int NKG = NCHUNK * CCH / 16;       // 16-channel groups over all chunks
  __shared__ __attribute__((aligned(16))) float tile[(TH + 2) * (kTW + 2) * LDP];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int tiles_x = (a.W + kTW - 1) / kTW;
  const int ntile = tiles_x * ((a.H + TH - 1) / TH);
  const int t = xcd_tile(blockIdx.x, ntile);
  const int ty0 = (t / tiles_x) * TH, tx0 = (t % tiles_x) * kTW;
  const int obase = blockIdx.y * OB;

  f32x4 acc[PB][OB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = zero4();

  const float* src0 = a.src0;
  const float* src1 = a.src1;
  if (a.sel != nullptr && *a.sel != 0u) {
    if (a.alt0 != nullptr) src0 = a.alt0;
    if (a.alt1 != nullptr) src1 = a.alt1;
  }

#pragma unroll
  for (int ch = 0; ch < NCHUNK; ++ch) {
    const float* src = ch == 0 ? src0 : src1;
    if (ch) __syncthreads();
    constexpr int V = CCH / 4;
    constexpr int NV = (TH + 2) * (kTW + 2) * V;
    for (int idx = threadIdx.x; idx < NV; idx += 256) {
      const int pix = idx / V, v = idx - pix * V;
      const int ly = pix / (kTW + 2), lx = pix - ly * (kTW + 2);
      const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
      f32x4 val = zero4();
      if (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
        val = ld4(src + ((size_t)gy * a.W + gx) * CCH + 4 * v);
      st4(&tile[pix * LDP + 4 * v], val);
    }
    __syncthreads();

    // (tap, 16-channel group) steps, software-pipelined: the A fragments (global) and
    // B fragments (LDS) of step i+1 are in flight while the MFMAs of step i issue.
    constexpr int NCG = CCH / 16;
    constexpr int NIT = 9 * NCG;
    const f32x4* wbase = a.wfrag + ((size_t)(ch * NCG) * a.obtot + obase) * 64 + lane;
    const size_t wstride_tap = (size_t)NKG * a.obtot * 64;
    const float* tbase = &tile[((wave * PB) * (kTW + 2) + j) * LDP + 4 * q];
    f32x4 wa[OB], xb[PB];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) wa[ob] = wbase[ob * 64];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) xb[pb] = ld4(tbase + pb * (kTW + 2) * LDP);
#pragma unroll 3
    for (int it = 0; it < NIT; ++it) {
      f32x4 wn[OB], xn[PB];
      if (it + 1 < NIT) {
        const int tap = (it + 1) / NCG, cg = (it + 1) - tap * NCG;
        const int dy = tap / 3, dx = tap - 3 * dy;
        const f32x4* wp = wbase + tap * wstride_tap + (size_t)cg * a.obtot * 64;
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) wn[ob] = wp[ob * 64];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          xn[pb] = ld4(tbase + ((pb + dy) * (kTW + 2) + dx) * LDP + 16 * cg);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = mfma4(wa[ob][kk], xb[pb][kk], acc[pb][ob]);
      if (it + 1 < NIT) {
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) wa[ob] = wn[ob];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) xb[pb] = xn[pb];
      }
    }
  }

#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int gy = ty0 + wave * PB + pb, gx = tx0 + j;
    if (gy >= a.H || gx >= a.W) continue;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = (obase + ob) * 16 + 4 * q;
      f32x4 v = acc[pb][ob] + ld4(a.bias + row);
      if (EPI == EPI_LRELU) {
        v = f32x4{lrelu(v[0]), lrelu(v[1]), lrelu(v[2]), lrelu(v[3])};
        st4(a.dst + ((size_t)gy * a.W + gx) * a.ldy + row, v);
      } else if (EPI == EPI_RES) {
        float* p = a.dst + ((size_t)gy * a.W + gx) * a.ldy + row;
        v += ld4(a.res + ((size_t)gy * a.W + gx) * a.ldy + row);
        st4(p, v);
      } else if (EPI == EPI_OFFSET) {
        float* p = a.dst + ((size_t)gy * a.W + gx) * a.ldy + row;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = row + r;
          if (o < a.cout) p[r] = o >= a.sig_lo ? sigmoidf(v[r]) : v[r];
        }
      } else {  // EPI_SHUFFLE: A row 16*ob + t is channel 16*(ob/4) + t at sub-pixel ob%4
        const int obg = obase + ob;
        const int sp = obg & 3, c = 16 * (obg >> 2) + 4 * q;
        const int Y = 2 * gy + (sp >> 1), X = 2 * gx + (sp & 1);
        v = f32x4{lrelu(v[0]), lrelu(v[1]), lrelu(v[2]), lrelu(v[3])};
        st4(a.dst + ((size_t)Y * (2 * a.W) + X) * a.ccout + c, v);
      }
    }
  }
}

// ---- modulated deformable conv, stride 1, pad 1, 3x3, over cat(fa, fb) ----
struct DcnArgs {
  const float* fa;
  const float* fb;
  const uint32_t* sel;
  const float* offs;
  const f32x4* wfrag;
  const float* bias;
  float* dst;
  int H, W, ldo, groups, obtot;
};

template <int C, int PB>
__global__ __launch_bounds__(256) void k_dcn(DcnArgs a) {
  constexpr int TH = 4 * PB;
  constexpr int OB = C / 16;
  constexpr int NKG = 2 * C / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;
  const int tiles_x = (a.W + kTW - 1) / kTW;
  const int ntile = tiles_x * ((a.H + TH - 1) / TH);
  const int t = xcd_tile(blockIdx.x, ntile);
  const int ty0 = (t / tiles_x) * TH, tx0 = (t % tiles_x) * kTW;
  const int cpg = 2 * C / a.groups;          // channels per offset group
  const int G = a.groups;
  const float* fb = (a.sel != nullptr && *a.sel != 0u) ? a.fa : a.fb;

  f32x4 acc[PB][OB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = zero4();

  // per-pixel offset rows (clamped for rows/columns past the image; results discarded)
  const float* orow[PB];
  int gys[PB];
  const int gx = tx0 + j;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    gys[pb] = ty0 + wave * PB + pb;
    orow[pb] = a.offs + ((size_t)min(gys[pb], a.H - 1) * a.W + min(gx, a.W - 1)) * a.ldo;
  }
  const float hmax = (float)a.H, wmax = (float)a.W;

  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap - 3 * (tap / 3);
#pragma unroll 2
    for (int kg = 0; kg < NKG; ++kg) {
      const int cgl = 16 * kg + 4 * q;                 // channel in cat(fa, fb)
      const float* src = cgl < C ? a.fa : fb;
      const int cl = cgl < C ? cgl : cgl - C;
      const int g = cgl / cpg;
      const f32x4* wp = a.wfrag + ((size_t)(tap * NKG + kg) * a.obtot) * 64 + lane;
      f32x4 wa[OB];
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) wa[ob] = wp[ob * 64];
      f32x4 xb[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        const float dyo = orow[pb][2 * (9 * g + tap)];
        const float dxo = orow[pb][2 * (9 * g + tap) + 1];
        const float m = orow[pb][18 * G + 9 * g + tap];
        // positions beyond one pixel outside the map sample only zeros; clamp so the
        // integer conversion below stays defined for any offset value
        const float py = fminf(fmaxf((float)(gys[pb] + ky - 1) + dyo, -2.0f), hmax + 1.0f);
        const float px = fminf(fmaxf((float)(gx + kx - 1) + dxo, -2.0f), wmax + 1.0f);
        const float y0f = floorf(py), x0f = floorf(px);
        const float ly = py - y0f, lx = px - x0f;
        const int y0 = (int)y0f, x0 = (int)x0f;
        f32x4 v = zero4();
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const int yy = y0 + cy;
          const float wy = cy ? ly : 1.0f - ly;
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const int xx = x0 + cx;
            const float wx = cx ? lx : 1.0f - lx;
            if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W)
              v += (wy * wx) * ld4(src + ((size_t)yy * a.W + xx) * C + cl);
          }
        }
        xb[pb] = v * m;
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) acc[pb][ob] = mfma4(wa[ob][kk], xb[pb][kk], acc[pb][ob]);
    }
  }

#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    if (gys[pb] >= a.H || gx >= a.W) continue;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int row = ob * 16 + 4 * q;
      f32x4 v = acc[pb][ob] + ld4(a.bias + row);
      v = f32x4{lrelu(v[0]), lrelu(v[1]), lrelu(v[2]), lrelu(v[3])};
      st4(a.dst + ((size_t)gys[pb] * a.W + gx) * C + row, v);
    }
  }
}

// ---- first conv 3 -> C on the vector ALUs: planar RGB in, NHWC out, LReLU ----
// blockIdx.y selects 16 output channels, so every weight read is uniform (scalar loads).
__global__ __launch_bounds__(256) void k_conv_in(const float* __restrict__ rgb,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ dst, int H, int W, int C) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= H * W) return;
  const int y = p / W, x = p - y * W;
  const int o0 = blockIdx.y * 16;
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
  float out[16];
#pragma unroll
  for (int o = 0; o < 16; ++o) {
    float s = b[o0 + o];
    const float* wo = w + (size_t)(o0 + o) * 27;
#pragma unroll
    for (int k = 0; k < 27; ++k) s = fmaf(wo[k], in[k], s);
    out[o] = lrelu(s);
  }
  float* d = dst + (size_t)p * C + o0;
#pragma unroll
  for (int v = 0; v < 4; ++v) st4(d + 4 * v, f32x4{out[4 * v], out[4 * v + 1], out[4 * v + 2], out[4 * v + 3]});
}

// ---- HR conv C -> 3 plus the bilinear x2 base, planar RGB out ----
// The thin output conv is computed as "tap responses": R[3*tap + o][p] =
// sum_c w[o][c][tap] U[c][p] is a 27-row (padded to 32) by C product on MFMA, taken over
// every pixel of a 16x16 output tile and its one-pixel halo and kept in LDS; each
// output pixel then sums the nine responses of its shifted neighbours:
//   out[o][p] = b[o] + sum_tap R[3*tap + o][p + delta_tap] + base[o][p].
// Pixels outside the map have U = 0, hence R = 0: the conv's zero padding.
// tsel: 0 -> base of frame a, 1 -> frame b, 2 -> the mean of both.
__device__ __forceinline__ float up2_sample(const float* pl, int H, int W, int Y, int X) {
  const int i = Y >> 1, jx = X >> 1;
  const int i2 = (Y & 1) ? min(i + 1, H - 1) : max(i - 1, 0);
  const int j2 = (X & 1) ? min(jx + 1, W - 1) : max(jx - 1, 0);
  const float r0 = 0.75f * pl[(size_t)i * W + jx] + 0.25f * pl[(size_t)i2 * W + jx];
  const float r1 = 0.75f * pl[(size_t)i * W + j2] + 0.25f * pl[(size_t)i2 * W + j2];
  return 0.75f * r0 + 0.25f * r1;
}

struct HrArgs {
  const float* u;        // [2H][2W][C]
  const f32x4* wfrag;    // [C/16][2][64] fragments of the 32 x C response matrix
  const float* bias;     // [3]
  const float* rgb_a;
  const float* rgb_b;
  const uint32_t* sel;
  float* dst;            // [3][2H][2W]
  int H, W, tsel;
};

template <int C>
__global__ __launch_bounds__(256) void k_hr(HrArgs a) {
  constexpr int T = 16, RW = T + 2, NP = RW * RW, NPB = (NP + 15) / 16, LDR = 33;
  constexpr int NCG = C / 16;
  __shared__ float R[NPB * 16 * LDR];
  const int H2 = 2 * a.H, W2 = 2 * a.W;
  const int tiles_x = (W2 + T - 1) / T;
  const int ntile = tiles_x * ((H2 + T - 1) / T);
  const int t = xcd_tile(blockIdx.x, ntile);
  const int ty0 = (t / tiles_x) * T, tx0 = (t % tiles_x) * T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, j = lane & 15;

  f32x4 wa[NCG][2];
#pragma unroll
  for (int cg = 0; cg < NCG; ++cg) {
    wa[cg][0] = a.wfrag[(cg * 2 + 0) * 64 + lane];
    wa[cg][1] = a.wfrag[(cg * 2 + 1) * 64 + lane];
  }
  for (int pbk = wave; pbk < NPB; pbk += 4) {
    const int p = pbk * 16 + j;
    const int ry = p / RW, rx = p - ry * RW;
    const int Y = ty0 + ry - 1, X = tx0 + rx - 1;
    const bool ok = p < NP && Y >= 0 && Y < H2 && X >= 0 && X < W2;
    const float* up = a.u + ((size_t)(ok ? Y : 0) * W2 + (ok ? X : 0)) * C + 4 * q;
    f32x4 acc0 = zero4(), acc1 = zero4();
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      const f32x4 xb = ok ? ld4(up + 16 * cg) : zero4();
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        acc0 = mfma4(wa[cg][0][kk], xb[kk], acc0);
        acc1 = mfma4(wa[cg][1][kk], xb[kk], acc1);
      }
    }
    float* rp = &R[p * LDR];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      rp[4 * q + r] = acc0[r];
      rp[16 + 4 * q + r] = acc1[r];
    }
  }
  __syncthreads();
  const int ly = threadIdx.x / T, lx = threadIdx.x - ly * T;
  const int Y = ty0 + ly, X = tx0 + lx;
  if (Y >= H2 || X >= W2) return;
  float s0 = a.bias[0], s1 = a.bias[1], s2 = a.bias[2];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap - 3 * dy;
    const float* rp = &R[((ly + dy) * RW + lx + dx) * LDR + 3 * tap];
    s0 += rp[0];
    s1 += rp[1];
    s2 += rp[2];
  }
  const size_t lpl = (size_t)a.H * a.W, hpl = (size_t)H2 * W2;
  const float* rb = (a.sel != nullptr && *a.sel != 0u) ? a.rgb_a : a.rgb_b;
  float base[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (a.tsel == 0) base[c] = up2_sample(a.rgb_a + c * lpl, a.H, a.W, Y, X);
    else if (a.tsel == 1) base[c] = up2_sample(rb + c * lpl, a.H, a.W, Y, X);
    else base[c] = 0.5f * (up2_sample(a.rgb_a + c * lpl, a.H, a.W, Y, X) + up2_sample(rb + c * lpl, a.H, a.W, Y, X));
  }
  a.dst[(size_t)Y * W2 + X] = s0 + base[0];
  a.dst[hpl + (size_t)Y * W2 + X] = s1 + base[1];
  a.dst[2 * hpl + (size_t)Y * W2 + X] = s2 + base[2];
}

template <int CCH, int NCHUNK, int OB, int PB, int EPI>
hipError_t run_conv(const ConvArgs& a, hipStream_t s) {
  constexpr int TH = 4 * PB;
  const int ntile = ((a.W + kTW - 1) / kTW) * ((a.H + TH - 1) / TH);
  const dim3 grid(ntile, a.obtot / OB);
  hipLaunchKernelGGL((k_conv3x3<CCH, NCHUNK, OB, PB, EPI>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int CCH, int NCHUNK>
hipError_t dispatch_epi(const ConvArgs& a, int epi, hipStream_t s) {
  constexpr int PB = 2;
  switch (epi) {
    case EPI_LRELU:
      if (a.obtot % 4 == 0) return run_conv<CCH, NCHUNK, 4, PB, EPI_LRELU>(a, s);
      return run_conv<CCH, NCHUNK, 2, PB, EPI_LRELU>(a, s);
    case EPI_RES:
      if (a.obtot % 4 == 0) return run_conv<CCH, NCHUNK, 4, PB, EPI_RES>(a, s);
      return run_conv<CCH, NCHUNK, 2, PB, EPI_RES>(a, s);
    case EPI_OFFSET:
      if (a.obtot % 7 == 0) return run_conv<CCH, NCHUNK, 7, PB, EPI_OFFSET>(a, s);
      if (a.obtot % 4 == 0) return run_conv<CCH, NCHUNK, 4, PB, EPI_OFFSET>(a, s);
      return run_conv<CCH, NCHUNK, 1, PB, EPI_OFFSET>(a, s);
    case EPI_SHUFFLE: return run_conv<CCH, NCHUNK, 8, PB, EPI_SHUFFLE>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_conv_in(const PlainConv& L, const float* rgb, float* dst, int H, int W,
                          hipStream_t s) {
  const dim3 grid((H * W + 255) / 256, L.cout / 16);
  hipLaunchKernelGGL(k_conv_in, grid, dim3(256), 0, s, rgb, L.w, L.b, dst, H, W, L.cout);
  return hipGetLastError();
}

hipError_t launch_conv(const PackedConv& L, int epi, const float* src0, const float* src1,
                       const uint32_t* sel, const float* alt0, const float* alt1,
                       const float* res, float* dst, int ldy, int H, int W, int sig_lo,
                       hipStream_t s) {
  ConvArgs a;
  a.src0 = src0;
  a.src1 = src1;
  a.sel = sel;
  a.alt0 = alt0;
  a.alt1 = alt1;
  a.wfrag = reinterpret_cast<const f32x4*>(L.frag);
  a.bias = L.bias;
  a.res = res;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.ldy = ldy;
  a.cout = L.cout;
  a.sig_lo = sig_lo;
  a.obtot = L.obtot;
  a.ccout = L.cout / 4;
  const int nchunk = src1 ? 2 : 1;
  const int cch = L.cin / nchunk;
  if (cch == 64 && nchunk == 1) return dispatch_epi<64, 1>(a, epi, s);
  if (cch == 64 && nchunk == 2) return dispatch_epi<64, 2>(a, epi, s);
  if (cch == 32 && nchunk == 1) return dispatch_epi<32, 1>(a, epi, s);
  if (cch == 32 && nchunk == 2) return dispatch_epi<32, 2>(a, epi, s);
  return hipErrorInvalidValue;
}

hipError_t launch_dcn(const PackedConv& L, const float* fa, const float* fb, const uint32_t* sel,
                      const float* offs, int ldo, int groups, float* dst, int H, int W,
                      hipStream_t s) {
  DcnArgs a;
  a.fa = fa;
  a.fb = fb;
  a.sel = sel;
  a.offs = offs;
  a.wfrag = reinterpret_cast<const f32x4*>(L.frag);
  a.bias = L.bias;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.ldo = ldo;
  a.groups = groups;
  a.obtot = L.obtot;
  constexpr int PB = 2;
  const int ntile = ((W + kTW - 1) / kTW) * ((H + 4 * PB - 1) / (4 * PB));
  if (L.cout == 64) hipLaunchKernelGGL((k_dcn<64, PB>), dim3(ntile), dim3(256), 0, s, a);
  else if (L.cout == 32) hipLaunchKernelGGL((k_dcn<32, PB>), dim3(ntile), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_hr(const PlainConv& L, const float* u, const float* rgb_a, const float* rgb_b,
                     const uint32_t* sel, int tsel, float* dst, int H, int W, hipStream_t s) {
  HrArgs a;
  a.u = u;
  a.wfrag = reinterpret_cast<const f32x4*>(L.w);
  a.bias = L.b;
  a.rgb_a = rgb_a;
  a.rgb_b = rgb_b;
  a.sel = sel;
  a.dst = dst;
  a.H = H;
  a.W = W;
  a.tsel = tsel;
  const int ntile = ((2 * W + 15) / 16) * ((2 * H + 15) / 16);
  if (L.cin == 64) hipLaunchKernelGGL((k_hr<64>), dim3(ntile), dim3(256), 0, s, a);
  else if (L.cin == 32) hipLaunchKernelGGL((k_hr<32>), dim3(ntile), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace nv

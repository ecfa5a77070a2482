// Host-side declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nv {

// One Y'CbCr frame as the kernels see it.  matrix: 709, 601 or 2020; full: full-range
// codes; centre: 4:2:0 chroma sited at the centre of its 2x2 luma block (else co-sited
// with the even luma column).
struct Frame {
  const void* p[3];
  int64_t pitch[3];   // bytes
  int w, h, bits, chroma;
  int matrix = 709, full = 0, centre = 0;
};

struct FrameOut {
  void* p[3];
  int64_t pitch[3];
  int w, h, bits, chroma;
  int matrix = 709, full = 0, centre = 0;
};

struct SceneRule {
  int mad_thresh_8bit, hist_num, hist_den, enable;
};

// Constants of the inverse (unpack) and forward (pack) matrices of one colourspace
// (matrix 709 / 601 / 2020, limited or full range) and bit depth; every derived
// coefficient is formed in double and rounded once.
struct Inv {
  float ys, yo, cs, co, rcr, bcb, gcb, gcr;
};
struct Fwd {
  float kr, kg, kb, cbs, crs, ys, yo, cs, co, maxc;
};
Inv make_inv(int bits, int matrix = 709, int full = 0);
Fwd make_fwd(int bits, int matrix = 709, int full = 0);

// ---- pixel-format stages (k_pixel.hip) ----
hipError_t launch_unpack(const Frame& f, float* rgb, int hp, int wp, hipStream_t s);
hipError_t launch_pack(const FrameOut& f, const float* rgb, int rh, int rw, hipStream_t s);
struct SceneJob;
// One frame's scene metric: accumulate, then decide (after a clear of job.sad / hist when
// `clear`; otherwise they must be zero, as a previous call with job.reset leaves them).
hipError_t launch_scene(const SceneJob& job, bool clear, hipStream_t s);

// ---- batched (multi-image, persistent) launches ----
// Each batched kernel walks a device table of jobs.  Job j owns the work items
// [item_begin_j, item_begin_{j+1}); count[0] is the number of jobs and count[1] the
// total number of items, both read on the device, so one captured graph serves any
// batch that fits the tables.  Blocks grid-stride over the items.
constexpr int kBatchGrid = 2048;          // persistent workgroups per batched launch
constexpr int kSceneRowsPerItem = 8;

struct UnpackJob {
  Frame f;
  Inv m;
  float* rgb;
  int hp, wp;
  int item_begin;
};

struct PackJob {
  FrameOut f;
  Fwd m;
  const float* rgb;
  int rh, rw;
  int item_begin;
};

// The scene metric of one frame.  sad / hist accumulate over the frame (zero at the
// start); the decision writes hd and cut and, when set, copies hist to hist_save and
// the SAD to sad_save.
struct SceneJob {
  Frame cur;
  const void* prev_y;          // previous frame's luma, or null for a stream's first frame
  int64_t prev_pitch;
  const uint32_t* hist_prev;
  uint64_t* sad;
  uint32_t* hist;              // histogram of cur (accumulator)
  uint32_t* hd;
  uint32_t* cut;
  uint32_t* hist_save;
  uint64_t* sad_save;
  void* luma_save;             // when set, the accumulate pass copies cur's luma rows there
  int64_t luma_save_pitch;
  SceneRule rule;
  int external;
  int reset;                   // single-frame launch: zero sad and hist after the decision
  int item_begin;              // batched launch: first item, in row chunks of kSceneRowsPerItem
};

inline int unpack_items(int hp, int wp) { return ((wp / 4) * hp + 255) / 256; }
inline int pack_items(int w, int h, int chroma) {
  const int n = chroma == 420 ? ((w / 2 + 3) / 4) * (h / 2) : ((w + 7) / 8) * h;
  return (n + 255) / 256;
}
inline int scene_items(int h) { return (h + kSceneRowsPerItem - 1) / kSceneRowsPerItem; }

hipError_t launch_unpack_batch(const UnpackJob* jobs, const int* count, hipStream_t s);
hipError_t launch_pack_batch(const PackJob* jobs, const int* count, hipStream_t s);
// count: {njobs, accumulate items}
hipError_t launch_scene_batch(const SceneJob* jobs, const int* count, hipStream_t s);

// ---- network (k_net.hip) ----
// DT_F8 (OCP e4m3) is an MFMA operand type only; FP8 layers read and write float16.
enum DType { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2, DT_F8 = 3 };

inline int dtype_bytes(int dt) { return dt == DT_F32 ? 4 : (dt == DT_F8 ? 1 : 2); }

// Packed weights of one conv for the MFMA kernels: fragment-ordered A operands in the
// MFMA type tc (16 bytes per lane, 32 for FP8), and the float bias per A row.  For the
// HR conv the fragments hold the 32 x C tap-response matrix.  FP8 layers also carry
// the per-row output scale (weight scale x activation scale) and the reciprocal
// activation scale, both in device memory so that recalibration needs no relaunch
// setup (captured graphs read the current values).
struct PackedConv {
  void* frag = nullptr;    // device
  void* frag32 = nullptr;  // device, 32-row fragments for the 32x32 MFMA form (16-bit bulk convs)
  float* bias = nullptr;   // device, obtot*16 floats
  float* oscale = nullptr; // device, obtot*16 floats (FP8 only)
  float* ainv = nullptr;   // device scalar (FP8 only)
  int cin = 0, cout = 0, obtot = 0, tc = DT_F32;
  int sv = 2, sh = 2;      // pixel-shuffle conv: sub-pixel rows and columns of its output
};

// The 3 -> C input conv runs on the vector ALUs with the plain OIHW layout.
struct PlainConv {
  float* w = nullptr;      // device
  float* b = nullptr;      // device
  int cin = 0, cout = 0;
};

enum ConvEpi { EPI_LRELU = 0, EPI_RES = 1, EPI_OFFSET = 2, EPI_SHUFFLE = 3 };
// Role of a conv: bulk (residual blocks, pixel-shuffle conv; storage = MFMA type), the
// offset head's first conv (two 16- or 32-bit inputs, float MFMA), its second conv (float).
enum ConvRole { CONV_BULK = 0, CONV_OFF1 = 1, CONV_OFF2 = 2 };

// Per-image arguments of a conv launch (one job of a batched launch).  When sel is
// non-null and *sel != 0 on the device, alt0 / alt1 (where non-null) replace src0 /
// src1 -- the device-side selection of a duplicated frame at a scene cut.
struct ConvImg {
  const void* src0;
  const void* src1;
  const uint32_t* sel;
  const void* alt0;
  const void* alt1;
  const void* res;
  void* dst;
  int H, W;
  int item_begin;
};

struct ConvInImg {
  const float* rgb;
  void* dst;
  int H, W;
  int item_begin;              // in 256-pixel blocks x (C/16) channel blocks
};

struct DcnImg {
  const void* fa;
  const void* fb;
  const uint32_t* sel;
  const float* offs;
  void* dst;
  int H, W;
  int item_begin;
};

// The output conv of one image: U is [sv H][sh W][C], the output R'G'B' [3][sv H][sh W].
struct HrImg {
  const void* u;
  const float* rgb_a;
  const float* rgb_b;
  const uint32_t* sel;
  float* dst;
  int H, W, tsel;
  int item_begin;
  int sv = 2, sh = 2;
};

// Tile shape of a bulk conv launch: rows per wave pb (1, 2, 4; a workgroup covers 4 pb
// rows), waves along the output blocks wo (1, 2; each wave then takes pb * wo rows and
// 1/wo of the workgroup's output blocks), and lw: the persistent form that keeps a
// 64-channel output group's weights in LDS (16-bit and FP8, pb 2 or 4, wo 1), packed
// in one int.
inline int tile_code(int pb, int wo, int lw = 0, int m32 = 0) {
  return pb | ((wo - 1) << 8) | (lw << 12) | (m32 << 13);
}
inline int tile_pb(int code) { return code & 0xFF; }
inline int tile_wo(int code) { return 1 + ((code >> 8) & 0xF); }
inline int tile_lw(int code) { return (code >> 12) & 1; }
// m32: 32x32x16 MFMA form (16-bit bulk convs with 64 input channels): each wave takes
// pb rows as pb / 2 blocks of 32 pixels (two rows of 16), pb = 2 or 4, wo = 1.
inline int tile_m32(int code) { return (code >> 13) & 1; }

// Static LDS of a bulk conv tile (MFMA type tc, cch input channels), and the current
// device's per-workgroup LDS limit; tiles above the limit are refused by the dispatch.
int bulk_tile_lds(int tc, int cch, int tile);
int lds_limit();
bool lds_weight_tiles();   // whether the LDS-resident-weight tiles are enabled

// Output blocks per workgroup chosen by the conv dispatch for a role / epilogue / MFMA
// type / tile code.
int conv_ob(int role, int epi, int obtot, int tc, int tile);

// One residual block, y = x + conv_b(LReLU(conv_a(x))), as one launch (16-bit maps,
// C = 64); im.src0 = x, im.dst = y (a different buffer), im.H / im.W.  Bit-identical to
// the two separate bulk-conv launches.
bool resblock_supported(const PackedConv& A, const PackedConv& Bc, int tin);
hipError_t launch_resblock(const PackedConv& A, const PackedConv& Bc, int tin, const ConvImg& im, hipStream_t s);
inline int conv_items(int H, int W, int pb, int nobg) {
  return ((W + 15) / 16) * ((H + 4 * pb - 1) / (4 * pb)) * nobg;
}
inline int hr_items(int H, int W, int sv = 2, int sh = 2) { return ((sh * W + 15) / 16) * ((sv * H + 15) / 16); }
// input conv: one item per run of 4096 / C consecutive pixels (all C channels)
inline int conv_in_items(int H, int W, int C) { return (H * W + 4096 / C - 1) / (4096 / C); }

hipError_t launch_conv_in(const PlainConv& L, int tout, const float* rgb, void* dst, int H, int W,
                          hipStream_t s);
// dst (and res) NHWC with channel stride ldy.  src1 only for CONV_OFF1.  pb = tile code
// of bulk convs (tile_code), 2 for the offset head.
hipError_t launch_conv(const PackedConv& L, int role, int epi, int tin, int pb, const ConvImg& im,
                       int ldy, int sig_lo, hipStream_t s);
hipError_t launch_dcn(const PackedConv& L, int tf, int pb, const DcnImg& im, int ldo, int groups,
                      hipStream_t s);
// DCN tile code: rows per wave (1, 2), plus kDcnWindow for the form that reads a phase's
// sampling corners from an LDS copy of their window (float and 16-bit maps with at least
// 8 channels per offset group for 16-bit; bit-identical to the plain form).
constexpr int kDcnWindow = 16;
inline bool dcn_window_supported(int tf, int tc, int C, int groups) {
  const int cpg = 2 * C / groups;
  return tc == tf && tf != DT_F8 && (tf == DT_F32 ? cpg >= 4 : cpg >= 8);
}
// kDcnStaged (one row per wave only): the plain form's gather and sample buffer with the
// corners read from an LDS copy of the phase's window (float and 16-bit maps with at least
// 8 channels per offset group; bit-identical to the plain form).
constexpr int kDcnStaged = 32;
inline bool dcn_staged_supported(int tf, int tc, int C, int groups) {
  const int cpg = 2 * C / groups;
  return tc == tf && tf != DT_F8 && cpg >= 8 && (C == 32 || C == 64);
}
// HR conv C->3 plus the bilinear x2 base of frame a (tsel 0), b (1) or their mean (2).
hipError_t launch_hr(const PackedConv& L, int tu, const HrImg& im, hipStream_t s);

// ---- feature pyramid (k_pyr.hip), NHWC maps of type t (float or 16-bit) ----
// dst (H2 x W2 x C) = the 2x2 block means of src (2 H2 x 2 W2 x C).
hipError_t launch_pool2(int t, const void* src, void* dst, int H2, int W2, int C, hipStream_t s);
// dst[y][x][c] += scale * (x2 bilinear resize of src)[y][x][c] for c < nch; dst H x W
// with channel stride ldd, src H/2 x W/2 with channel stride lds (H, W even).
hipError_t launch_up2_add(int t, void* dst, int ldd, const void* src, int lds, int H, int W, int nch, float scale,
                          hipStream_t s);

// FP8 calibration: folds max |x| over n elements of x (float16 or float) into
// *amax_bits (float bits, atomic max), and derives a layer's scales from it.
hipError_t launch_amax(int dt, const void* x, size_t n, uint32_t* amax_bits, hipStream_t s);
hipError_t launch_qscale(const uint32_t* amax_bits, const float* wscale, float* oscale, float* ainv, int rows,
                         hipStream_t s);

hipError_t launch_conv_in_batch(const PlainConv& L, int tout, const ConvInImg* jobs, const int* count,
                                hipStream_t s);
hipError_t launch_conv_batch(const PackedConv& L, int role, int epi, int tin, int pb,
                             const ConvImg* jobs, const int* count, int ldy, int sig_lo, hipStream_t s);
hipError_t launch_dcn_batch(const PackedConv& L, int tf, int pb, const DcnImg* jobs, const int* count,
                            int ldo, int groups, hipStream_t s);
hipError_t launch_hr_batch(const PackedConv& L, int tu, const HrImg* jobs, const int* count,
                           hipStream_t s);

}  // namespace nv

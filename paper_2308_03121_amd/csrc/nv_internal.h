// Host-side declarations shared by the library's translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace nv {

// One Y'CbCr frame as the kernels see it.
struct Frame {
  const void* p[3];
  int64_t pitch[3];   // bytes
  int w, h, bits, chroma;
};

struct FrameOut {
  void* p[3];
  int64_t pitch[3];
  int w, h, bits, chroma;
};

struct SceneRule {
  int mad_thresh_8bit, hist_num, hist_den, enable;
};

// ---- pixel-format stages (k_pixel.hip) ----
hipError_t launch_unpack(const Frame& f, float* rgb, int hp, int wp, hipStream_t s);
hipError_t launch_pack(const FrameOut& f, const float* rgb, int rh, int rw, hipStream_t s);
// prev may have null p[0] (first frame).  hist_prev may be null.
hipError_t launch_scene(const Frame& cur, const Frame* prev, const uint32_t* hist_prev,
                        const SceneRule& rule, int external_cut, uint64_t* sad,
                        uint32_t* hist, uint32_t* hd, uint32_t* cut, hipStream_t s);

// ---- network (k_net.hip) ----
// Packed weights of one 3x3 conv for the MFMA kernels: fragment-ordered A operands
// [tap][kgroup][oblock][lane] x 4 floats, and the bias per A row.
struct PackedConv {
  float* frag = nullptr;   // device
  float* bias = nullptr;   // device, obtot*16 floats
  int cin = 0, cout = 0, obtot = 0;
};

// Small convs done on the vector ALUs keep their plain layout.
struct PlainConv {
  float* w = nullptr;      // device
  float* b = nullptr;      // device
  int cin = 0, cout = 0;
};

enum ConvEpi { EPI_LRELU = 0, EPI_RES = 1, EPI_OFFSET = 2, EPI_SHUFFLE = 3 };

hipError_t launch_conv_in(const PlainConv& L, const float* rgb, float* dst, int H, int W,
                          hipStream_t s);
// dst (and res) NHWC with channel stride ldy.  src1 may be null (single source).  When
// sel is non-null and *sel != 0 on the device, alt0 / alt1 (where non-null) replace
// src0 / src1 -- the device-side selection of a duplicated frame at a scene cut.
hipError_t launch_conv(const PackedConv& L, int epi, const float* src0, const float* src1,
                       const uint32_t* sel, const float* alt0, const float* alt1,
                       const float* res, float* dst, int ldy, int H, int W, int sig_lo,
                       hipStream_t s);
hipError_t launch_dcn(const PackedConv& L, const float* fa, const float* fb,
                      const uint32_t* sel, const float* offs, int ldo, int groups,
                      float* dst, int H, int W, hipStream_t s);
// HR conv C->3 plus the bilinear x2 base of frame a (tb = 0), b (tb = 1) or their mean.
hipError_t launch_hr(const PlainConv& L, const float* u, const float* rgb_a, const float* rgb_b,
                     const uint32_t* sel, int tsel, float* dst, int H, int W, hipStream_t s);

}  // namespace nv

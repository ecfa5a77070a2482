// Host runtime and C-ABI of the enhancement library: argument validation, weight
// repacking, the per-context workspace, the frame-group pipeline and clip streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <type_traits>
#include <new>
#include <string>
#include <vector>

#include "../../include/nnvisr.h"
#include "nv_internal.h"

using namespace nv;

// ------------------------------------------------------------------ errors ----

static thread_local std::string g_err;

static nv_status fail(nv_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                 \
  } while (0)

extern "C" const char* nv_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ config ----

namespace {

constexpr int kMaxDim = 16384;
constexpr int kCutRing = 1 << 16;   // device cut flags kept per stream (ring)
constexpr int kClipMaxPositions = 64;   // frame-store positions of a general-n clip (n b + b)

struct LayerSpec {
  const char* name;
  int cout, cin;
  int level = 1;   // feature-pyramid level of a "down" conv or a fusion layer
};

// Task of a network (section 3.2): scale factors and the Interpolation (with Extra
// frame) and Double frame flags.
int scale_h(const nv_net_config& c) { return c.scale; }
int scale_v(const nv_net_config& c) { return c.scale_v ? c.scale_v : c.scale; }
bool interpolating(const nv_net_config& c) { return (c.flags & NV_FLAG_INTERP) != 0; }
bool doubling(const nv_net_config& c) { return (c.flags & NV_FLAG_DOUBLE) != 0; }
bool default_task(const nv_net_config& c) {
  return scale_h(c) == 2 && scale_v(c) == 2 && interpolating(c) && doubling(c);
}
// Feature-pyramid levels (section 3.1: the extract stage's output); 0 reads as 1.
int pyramid_levels(const nv_net_config& c) { return c.levels > 1 ? c.levels : 1; }
constexpr int kMaxLevels = 4;   // level 4 is 1/8 of a padded frame (a multiple of 8)

std::vector<LayerSpec> layer_specs(const nv_net_config& c) {
  const int C = c.channels, G = c.offset_groups;
  std::vector<LayerSpec> v;
  v.push_back({"conv_in", C, 3});
  for (int r = 0; r < c.res_blocks; ++r) {
    v.push_back({"block.a", C, C});
    v.push_back({"block.b", C, C});
  }
  const int L = pyramid_levels(c);
  for (int l = 2; l <= L; ++l) v.push_back({"down", C, C, l});
  if (interpolating(c)) {
    for (int l = 1; l <= L; ++l) {
      v.push_back({"off1", C, 2 * C, l});
      v.push_back({"off2", 27 * G, C, l});
      v.push_back({"dcn", C, 2 * C, l});
    }
  }
  v.push_back({"up", scale_v(c) * scale_h(c) * C, C});
  v.push_back({"hr", 3, C});
  return v;
}

nv_status check_config(const nv_net_config* c) {
  if (!c) return fail(NV_E_INVALID, "config is NULL");
  if (c->channels != 32 && c->channels != 64)
    return fail(c->channels > 0 && c->channels % 32 == 0 ? NV_E_UNSUPPORTED : NV_E_INVALID,
                "channels must be 32 or 64 (got %d)", c->channels);
  if (c->res_blocks < 0 || c->res_blocks > 64)
    return fail(NV_E_INVALID, "res_blocks must be in [0, 64] (got %d)", c->res_blocks);
  const int G = c->offset_groups;
  if (G <= 0 || G % 2 != 0 || (2 * c->channels) % G != 0 || ((2 * c->channels) / G) % 4 != 0)
    return fail(NV_E_INVALID,
                "offset_groups must be even and split 2C into groups of a multiple of 4 channels");
  if (c->scale != 1 && c->scale != 2) return fail(NV_E_UNSUPPORTED, "scale must be 1 or 2 (got %d)", c->scale);
  if (c->scale_v != 0 && c->scale_v != 1 && c->scale_v != 2)
    return fail(NV_E_UNSUPPORTED, "scale_v must be 0, 1 or 2 (got %d)", c->scale_v);
  if (c->align != 8) return fail(NV_E_UNSUPPORTED, "only align 8 is implemented");
  const uint32_t task = c->flags & ~(uint32_t)(NV_FLAG_HEAD_FP32 | NV_FLAG_FP8_FUSION);
  if (task != (NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE) && task != (NV_FLAG_INTERP | NV_FLAG_EXTRA) &&
      task != 0)
    return fail(NV_E_UNSUPPORTED, "flags must be Interpolation|Extra frame[|Double frame] or none");
  if (task == (NV_FLAG_INTERP | NV_FLAG_EXTRA) && (c->scale != 1 || scale_v(*c) != 1))
    return fail(NV_E_INVALID, "without Double frame the input frames pass through: scale must be 1");
  if ((c->flags & NV_FLAG_FP8_FUSION) && c->precision != NV_FP8_E4M3)
    return fail(NV_E_INVALID, "NV_FLAG_FP8_FUSION needs NV_FP8_E4M3 precision");
  if (c->precision < NV_FP32 || c->precision > NV_FP8_E4M3)
    return fail(NV_E_INVALID, "precision %d is not an nv_precision", c->precision);
  if (c->precision == NV_FP8_E4M3 && c->channels != 64)
    return fail(NV_E_UNSUPPORTED, "FP8 precision is implemented for 64 channels");
  if (c->precision == NV_FP8_E4M3 && !default_task(*c))
    return fail(NV_E_UNSUPPORTED, "FP8 precision is implemented for the x2 space-time task");
  if (c->matrix != NV_MATRIX_BT709 && c->matrix != NV_MATRIX_BT601 && c->matrix != NV_MATRIX_BT2020)
    return fail(NV_E_INVALID, "matrix %d is not an NV_MATRIX_* value", c->matrix);
  if (c->range != NV_RANGE_LIMITED && c->range != NV_RANGE_FULL)
    return fail(NV_E_INVALID, "range %d is not an NV_RANGE_* value", c->range);
  if (c->levels < 0 || c->levels > kMaxLevels)
    return fail(NV_E_INVALID, "levels must be in [0, %d] (got %d)", kMaxLevels, c->levels);
  if (pyramid_levels(*c) > 1 && !interpolating(*c))
    return fail(NV_E_INVALID, "a feature pyramid needs an interpolating network (it feeds the alignment)");
  if (pyramid_levels(*c) > 1 && c->precision == NV_FP8_E4M3)
    return fail(NV_E_UNSUPPORTED, "FP8 precision is implemented for one pyramid level");
  return NV_OK;
}

size_t weight_count(const nv_net_config& c) {
  size_t n = 0;
  for (const auto& L : layer_specs(c)) n += (size_t)L.cout * L.cin * 9 + L.cout;
  return n;
}

nv_status check_format(const nv_format* f, const char* what) {
  if (!f) return fail(NV_E_INVALID, "%s format is NULL", what);
  if (f->bits != 8 && f->bits != 10) return fail(NV_E_INVALID, "%s: bits must be 8 or 10", what);
  if (f->chroma != 420 && f->chroma != 444) return fail(NV_E_INVALID, "%s: chroma must be 420 or 444", what);
  if (f->width <= 0 || f->height <= 0 || f->width > kMaxDim || f->height > kMaxDim)
    return fail(NV_E_INVALID, "%s: size %dx%d out of range", what, f->width, f->height);
  if (f->chroma == 420 && ((f->width | f->height) & 1))
    return fail(NV_E_INVALID, "%s: 4:2:0 needs even width and height", what);
  if (f->matrix != NV_MATRIX_BT709 && f->matrix != NV_MATRIX_BT601 && f->matrix != NV_MATRIX_BT2020)
    return fail(NV_E_INVALID, "%s: matrix %d is not an NV_MATRIX_* value", what, f->matrix);
  if (f->range != NV_RANGE_LIMITED && f->range != NV_RANGE_FULL)
    return fail(NV_E_INVALID, "%s: range %d is not an NV_RANGE_* value", what, f->range);
  if (f->chroma_loc != NV_SITING_LEFT && f->chroma_loc != NV_SITING_CENTER)
    return fail(NV_E_INVALID, "%s: chroma_loc %d is not an NV_SITING_* value", what, f->chroma_loc);
  return NV_OK;
}

int matrix_number(int m) { return m == NV_MATRIX_BT601 ? 601 : (m == NV_MATRIX_BT2020 ? 2020 : 709); }

nv_status check_planes(const nv_format* f, const nv_planes* p, const char* what) {
  if (!p) return fail(NV_E_INVALID, "%s planes are NULL", what);
  const int bps = f->bits == 8 ? 1 : 2;
  for (int i = 0; i < 3; ++i) {
    const int w = (i == 0 || f->chroma == 444) ? f->width : f->width / 2;
    if (!p->data[i]) return fail(NV_E_INVALID, "%s plane %d is NULL", what, i);
    if (p->pitch_bytes[i] < (int64_t)w * bps)
      return fail(NV_E_INVALID, "%s plane %d pitch %lld < %d bytes", what, i,
                  (long long)p->pitch_bytes[i], w * bps);
    if (bps == 2 && ((reinterpret_cast<uintptr_t>(p->data[i]) | (uintptr_t)p->pitch_bytes[i]) & 1))
      return fail(NV_E_INVALID, "%s plane %d: 16-bit samples must be 2-byte aligned", what, i);
  }
  return NV_OK;
}

Frame to_frame(const nv_format* f, const nv_planes* p) {
  Frame r;
  for (int i = 0; i < 3; ++i) {
    r.p[i] = p ? p->data[i] : nullptr;
    r.pitch[i] = p ? p->pitch_bytes[i] : 0;
  }
  r.w = f->width;
  r.h = f->height;
  r.bits = f->bits;
  r.chroma = f->chroma;
  r.matrix = matrix_number(f->matrix);
  r.full = f->range == NV_RANGE_FULL;
  r.centre = f->chroma == 420 && f->chroma_loc == NV_SITING_CENTER;
  return r;
}

FrameOut to_frame_out(const nv_format* f, const nv_planes* p) {
  FrameOut r;
  for (int i = 0; i < 3; ++i) {
    r.p[i] = p->data[i];
    r.pitch[i] = p->pitch_bytes[i];
  }
  r.w = f->width;
  r.h = f->height;
  r.bits = f->bits;
  r.chroma = f->chroma;
  r.matrix = matrix_number(f->matrix);
  r.full = f->range == NV_RANGE_FULL;
  r.centre = f->chroma == 420 && f->chroma_loc == NV_SITING_CENTER;
  return r;
}

int round_up(int v, int a) { return (v + a - 1) / a * a; }
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Every device allocation of the library goes through here.  Test hook: when the
// environment variable NNVISR_FAULT_ALLOC_MIN_BYTES holds a positive number, requests
// of at least that many bytes fail as out of memory (read at every call, so a test can
// switch it on and off around one call).
hipError_t dev_malloc(void** p, size_t bytes) {
  if (const char* f = getenv("NNVISR_FAULT_ALLOC_MIN_BYTES")) {
    const long long lim = atoll(f);
    if (lim > 0 && bytes >= (size_t)lim) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(p, bytes);
}

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
  return dev_malloc(reinterpret_cast<void**>(p), count * sizeof(T) > 0 ? count * sizeof(T) : 16);
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

// ------------------------------------------------------- static scratch ----

// Device scratch of the allocation-free group entry point (nv_enhance_group_static):
// one copy per device, allocated by the runtime with the code object and held until the
// process ends.  In host code the array's name is not a device address; the address of
// each device's copy comes from hipGetSymbolAddress at context creation (g_scratch_addr)
// and only that is passed to kernels.
static __device__ __align__(256) unsigned char g_static_scratch[NV_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Looks up the device address of the scratch array on `device`, the current device,
// once per device.
nv_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(NV_E_UNSUPPORTED, "device %d (at most %d)", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[device]) return NV_OK;
  void* p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(g_static_scratch)));
  if (!p) return fail(NV_E_DEVICE, "no device address for the static scratch on device %d", device);
  g_scratch_addr[device] = p;
  return NV_OK;
}

void* scratch_addr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_addr[device] : nullptr;
}

}  // namespace

// ------------------------------------------------------------------ context ----

struct Workspace {
  int hp = 0, wp = 0;
  void* t0 = nullptr;     // extract temporaries [hp][wp][C]      feature type
  float* o1 = nullptr;    // offset-head hidden  [hp][wp][C]      float
  float* offs = nullptr;  // offsets + mask      [hp][wp][ldo]    float
  void* fmid = nullptr;   // aligned features    [hp][wp][C]      feature type
  void* u = nullptr;      // HR features         [2hp][2wp][C]    feature type
  float* hr = nullptr;    // HR RGB              [3][2hp][2wp]    float
  float* rgb[2] = {nullptr, nullptr};  // group inputs [3][hp][wp]
  void* feat[2] = {nullptr, nullptr};  // group features: every pyramid level, level 1 first
  float* offs_lv = nullptr;  // pyramid levels 2..L: offsets + mask, level after level
  void* fmid_lv = nullptr;   // pyramid levels 2..L: aligned features, level after level
  void* u2 = nullptr;        // the t = 0 output's HR features and R'G'B' while it runs
  float* hr2 = nullptr;      // beside the alignment (null: no overlap)
  size_t bytes = 0;
};

// Orders device work that reuses one set of buffers (the context workspace, or one clip
// stream's ring and scene state) across the HIP streams a caller uses: the event
// recorded after the last call that touched the buffers, and the stream it ran on.  A
// call on another HIP stream first makes that stream wait for the event; calls on the
// same stream are ordered by the stream itself.
struct Order {
  hipEvent_t ev = nullptr;
  hipStream_t last = nullptr;
  bool any = false;
};

// Launch timing: a pair of HIP events around each launch while enabled.
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};

// Tile shapes of the kernels that have several (bulk convs: tile codes, see tile_code;
// DCN: rows per wave); the autotuner may change
// them per context (see nv_autotune).
struct Tuning {
  int pb_block = 2, pb_up = 2, pb_dcn = 2;
  int off1 = 2, off2 = 2;   // offset-head tile codes (split head: three shapes)
  int fused = 0;            // residual blocks as one launch where supported (1) or as two
};

struct BatchState;
static void batch_release(BatchState* b);

struct nv_context {
  int device = 0;
  Profiler prof;
  Tuning tune;
  BatchState* batch = nullptr;
  nv_net_config cfg{};
  int C = 0, G = 0, ldo = 0;
  int sv = 2, sh = 2;               // scale factors of the task (rows, columns)
  bool interp = true, dbl = true;   // Interpolation (with Extra frame), Double frame
  int ft = DT_F32;                  // feature storage type
  int bt = DT_F32;                  // MFMA type of the residual-block convs
  int ut = DT_F32;                  // MFMA type of the DCN contraction and the pixel-shuffle conv
  PlainConv conv_in;
  std::vector<PackedConv> blocks;   // a, b per residual block
  PackedConv off1, off2, dcn, up, hr;
  // feature pyramid: levels L, and for level l = 2..L (index l - 2) the conv after the
  // 2x2 mean pool and the level's offset head and DCN
  // side stream for the t = 0 output of a group, which needs no alignment and runs
  // beside it (fork / join events on the caller's stream)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int levels = 1;
  std::vector<PackedConv> down;
  struct LevelFusion {
    PackedConv off1, off2, dcn;
  };
  std::vector<LevelFusion> lvf;
  // FP8: quantised layers in calibration order (residual convs, dcn, up), each with
  // its per-row weight scales (device) and the running input max |x| (device, float
  // bits, one per layer); q_ready once scales were calibrated or set.
  std::vector<PackedConv*> q_layers;
  std::vector<float*> q_wscale;
  uint32_t* q_amax = nullptr;
  bool q_ready = false;
  bool calibrating = false;
  Workspace ws;
  Order ws_ord;                     // last use of ws
  std::vector<void*> allocs;
};

namespace {

// Feature pyramid geometry: level l (1-based) of an hp x wp map is (hp >> (l-1)) x
// (wp >> (l-1)) pixels (exact: padded sizes are multiples of 8 and L <= 4).  A frame's
// features hold the levels one after another, level 1 first, each [h_l][w_l][C]; the
// per-level offsets and aligned features of levels 2..L likewise, without level 1.
size_t level_px_before(int hp, int wp, int l) {
  size_t n = 0;
  for (int k = 1; k < l; ++k) n += (size_t)(hp >> (k - 1)) * (wp >> (k - 1));
  return n;
}
size_t feat_elems(const nv_context* ctx, int hp, int wp) {
  return (size_t)ctx->C * level_px_before(hp, wp, ctx->levels + 1);
}
size_t feat_bytes(const nv_context* ctx, int hp, int wp) {
  return feat_elems(ctx, hp, wp) * dtype_bytes(ctx->ft);
}
// Level l's map within a frame's feature buffer.
template <class P>
P* level_map(P* feat, const nv_context* ctx, int hp, int wp, int l) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(feat) +
                              (size_t)ctx->C * level_px_before(hp, wp, l) * dtype_bytes(ctx->ft));
}
// Pixels of levels 2..L (the extra per-level buffers of the fusion stage).
size_t upper_levels_px(const nv_context* ctx, int hp, int wp) {
  return level_px_before(hp, wp, ctx->levels + 1) - (size_t)hp * wp;
}

// float -> bfloat16 bits, round to nearest even (no NaN inputs occur in weights)
uint16_t to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

uint16_t to_f16_bits(float f) {
  _Float16 h = (_Float16)f;
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

// float -> OCP e4m3 (bias 7, 3 mantissa bits, largest finite 448, subnormal step 2^-9),
// round to nearest even, saturating to +-448.  The input is finite.
uint8_t to_e4m3_bits(float f) {
  const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
  const double a = std::fabs((double)f);
  if (a >= 448.0) return sign | 0x7E;
  int e = 0;
  std::frexp(a, &e);                       // a in [2^(e-1), 2^e)
  int E = a > 0.0 ? e - 1 : -6;
  if (E < -6) E = -6;                      // subnormals share the quantum of 2^-6
  const double quantum = std::ldexp(1.0, E - 3);
  const double v = std::nearbyint(a / quantum) * quantum;   // ties to even
  if (v < std::ldexp(1.0, -6)) return sign | (uint8_t)(v / std::ldexp(1.0, -9));   // subnormal (or 2^-6)
  int e2 = 0;
  std::frexp(v, &e2);
  const int Ev = e2 - 1;
  const int mant = (int)(v / std::ldexp(1.0, Ev - 3)) - 8;
  return sign | (uint8_t)((Ev + 7) << 3) | (uint8_t)mant;
}

// One lane fragment of an A operand: elements [c0, c0 + n) of row-vector getter g(c)
// in the MFMA type tc (n = 4 floats, 8 16-bit values or 32 e4m3 values).
template <class G>
void put_fragment(uint8_t* dst, int tc, int c0, G g) {
  if (tc == DT_F8) {
    for (int e = 0; e < 32; ++e) dst[e] = to_e4m3_bits(g(c0 + e));
  } else if (tc == DT_F32) {
    for (int e = 0; e < 4; ++e) {
      const float v = g(c0 + e);
      std::memcpy(dst + 4 * e, &v, 4);
    }
  } else {
    for (int e = 0; e < 8; ++e) {
      const uint16_t b = tc == DT_F16 ? to_f16_bits(g(c0 + e)) : to_bf16_bits(g(c0 + e));
      std::memcpy(dst + 2 * e, &b, 2);
    }
  }
}

// A-operand fragments of one conv for the MFMA kernels, 16 bytes per lane:
//   frag[((tap * NKG + kg) * obtot + ob) * 64 + lane]
//     = W[o = rowmap(16*ob + lane%16)][c = KG*kg + (KG/4)*(lane/16) + e][tap], e < KG/4
// with KG = 16 channels per group for float and 32 for 16-bit types, and
// bias[r] = b[rowmap(r)], zero for padded rows.  rowmap is the identity except for
// the pixel-shuffle conv (cout = r2 C for r2 = sv sh sub-pixels; r2 = 1: no reordering):
// its A row 16*ob + t carries channel 16*(ob % NB) + t of sub-pixel ob / NB (NB = C / 16
// row blocks per sub-pixel), i.e. original output channel r2*(16*(ob % NB) + t) + ob / NB,
// so that each group of NB blocks is one sub-pixel's whole channel vector.
nv_status pack_conv(nv_context* ctx, const float* w, const float* b, int cout, int cin,
                    int r2, int tc, PackedConv* out) {
  const int KG = tc == DT_F32 ? 16 : 32;
  const int obtot = (cout + 15) / 16;
  const int nkg = cin / KG;
  std::vector<uint8_t> frag((size_t)9 * nkg * obtot * 64 * 16, 0);
  std::vector<float> bias((size_t)obtot * 16, 0.0f);
  auto rowmap = [&](int r) -> int {
    if (r2 <= 1) return r;
    const int ob = r / 16, t = r % 16, nb = cout / (16 * r2);
    return r2 * (16 * (ob % nb) + t) + ob / nb;
  };
  for (int tap = 0; tap < 9; ++tap)
    for (int kg = 0; kg < nkg; ++kg)
      for (int ob = 0; ob < obtot; ++ob)
        for (int lane = 0; lane < 64; ++lane) {
          const int r = 16 * ob + lane % 16;
          if (r >= cout) continue;
          const int o = rowmap(r);
          const int c0 = KG * kg + (KG / 4) * (lane / 16);
          put_fragment(&frag[((((size_t)tap * nkg + kg) * obtot + ob) * 64 + lane) * 16], tc, c0,
                       [&](int c) { return w[((size_t)o * cin + c) * 9 + tap]; });
        }
  for (int r = 0; r < cout; ++r) bias[r] = b[rowmap(r)];
  out->cin = cin;
  out->cout = cout;
  out->obtot = obtot;
  out->tc = tc;
  HIP_TRY(dev_malloc((void**)&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  // 16-bit types: also the 32x32x16 MFMA A fragments, 16 bytes per lane:
  //   frag32[((tap * NKG16 + kg) * obtot32 + ob) * 64 + lane]
  //     = W[o = rowmap(32*ob + lane%32)][c = 16*kg + 8*(lane/32) + e][tap], e < 8
  if (tc != DT_F32 && cout % 32 == 0 && cin % 16 == 0) {
    const int ob32 = cout / 32, nkg16 = cin / 16;
    std::vector<uint8_t> f32x((size_t)9 * nkg16 * ob32 * 64 * 16, 0);
    for (int tap = 0; tap < 9; ++tap)
      for (int kg = 0; kg < nkg16; ++kg)
        for (int ob = 0; ob < ob32; ++ob)
          for (int lane = 0; lane < 64; ++lane) {
            const int o = rowmap(32 * ob + lane % 32);
            const int c0 = 16 * kg + 8 * (lane / 32);
            put_fragment(&f32x[((((size_t)tap * nkg16 + kg) * ob32 + ob) * 64 + lane) * 16], tc, c0,
                         [&](int c) { return w[((size_t)o * cin + c) * 9 + tap]; });
          }
    HIP_TRY(dev_malloc((void**)&out->frag32, f32x.size()));
    ctx->allocs.push_back(out->frag32);
    HIP_TRY(hipMemcpy(out->frag32, f32x.data(), f32x.size(), hipMemcpyHostToDevice));
  }
  HIP_TRY(dev_alloc(&out->bias, bias.size()));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

// Two-part float16 fragments of an offset-head conv (float-class head on float16 MFMA):
// with v = s * W[o][c % cin][tap] (s a power of two putting max |v| near 2^14), A
// position (kgroup, ob) holds two fragments, part 0 = f16(v) and part 1 = f16(v - f16(v)):
//   frag[((tap * NKG + kg) * 2*obtot + 2*ob + part) * 64 + lane], c = 32*kg + 8*(lane/16) + e
// over dup * cin input channels (dup = 2: the float input is staged as [hi | lo] and
// both halves meet the same weights).  oscale[r] = 1/s undoes the scaling.
nv_status pack_conv_split(nv_context* ctx, const float* w, const float* b, int cout, int cin, int dup,
                          PackedConv* out) {
  const int cin_v = cin * dup, KG = 32, nkg = cin_v / KG;
  const int obtot = (cout + 15) / 16;
  float m = 0.0f;
  for (size_t k = 0; k < (size_t)cout * cin * 9; ++k) m = std::max(m, std::fabs(w[k]));
  int e = m > 0.0f ? (int)std::floor(std::log2(16384.0 / m)) : 0;
  e = std::min(std::max(e, -14), 30);
  const float s = std::ldexp(1.0f, e);
  std::vector<uint8_t> frag((size_t)9 * nkg * 2 * obtot * 64 * 16, 0);
  for (int tap = 0; tap < 9; ++tap)
    for (int kg = 0; kg < nkg; ++kg)
      for (int ob = 0; ob < obtot; ++ob)
        for (int part = 0; part < 2; ++part)
          for (int lane = 0; lane < 64; ++lane) {
            const int o = 16 * ob + lane % 16;
            if (o >= cout) continue;
            const int c0 = KG * kg + (KG / 4) * (lane / 16);
            put_fragment(&frag[((((size_t)tap * nkg + kg) * 2 * obtot + 2 * ob + part) * 64 + lane) * 16],
                         DT_F16, c0, [&](int c) {
                           const float v = w[((size_t)o * cin + c % cin) * 9 + tap] * s;
                           const float hi = (float)(_Float16)v;
                           return part == 0 ? hi : v - hi;
                         });
          }
  std::vector<float> bias((size_t)obtot * 16, 0.0f), inv((size_t)obtot * 16, 1.0f / s);
  for (int r = 0; r < cout; ++r) bias[r] = b[r];
  out->cin = cin_v;
  out->cout = cout;
  out->obtot = obtot;
  out->tc = DT_F16;
  HIP_TRY(dev_malloc((void**)&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  HIP_TRY(dev_alloc(&out->bias, bias.size()));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(dev_alloc(&out->oscale, inv.size()));
  ctx->allocs.push_back(out->oscale);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->oscale, inv.data(), inv.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

// Per A row r (output channel rowmap(r)), the FP8 weight scale max |W| / 448.
std::vector<float> f8_row_scales(const float* w, int cout, int cin, int obtot, const std::function<int(int)>& rowmap) {
  std::vector<float> sc((size_t)obtot * 16, 1.0f);
  for (int r = 0; r < cout; ++r) {
    const int o = rowmap(r);
    float m = 0.0f;
    for (size_t k = 0; k < (size_t)cin * 9; ++k) m = std::max(m, std::fabs(w[(size_t)o * cin * 9 + k]));
    sc[r] = m > 0.0f ? m / 448.0f : 1.0f;
  }
  return sc;
}

// FP8 fragments of a 64-channel 3x3 conv (residual blocks, pixel-shuffle conv), 32 bytes
// per lane, five steps of two taps:
//   frag[(st * obtot + ob) * 64 + lane][e] = e4m3(W[o][c][tap] / s_w[r])
// with r = 16*ob + lane%16, o = rowmap(r), q = lane/16, tap = 2*st + q/2, c = 32*(q%2) + e,
// and zero where tap = 9.  wscale receives s_w per A row.
nv_status pack_conv_f8(nv_context* ctx, const float* w, const float* b, int cout, int cin, int r2,
                       PackedConv* out, std::vector<float>* wscale) {
  const int obtot = (cout + 15) / 16;
  std::vector<uint8_t> frag((size_t)5 * obtot * 64 * 32, 0);
  std::vector<float> bias((size_t)obtot * 16, 0.0f);
  auto rowmap = [&](int r) -> int {
    if (r2 <= 1) return r;
    const int ob = r / 16, t = r % 16, nb = cout / (16 * r2);
    return r2 * (16 * (ob % nb) + t) + ob / nb;
  };
  *wscale = f8_row_scales(w, cout, cin, obtot, rowmap);
  for (int st = 0; st < 5; ++st)
    for (int ob = 0; ob < obtot; ++ob)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = 16 * ob + lane % 16, q = lane / 16;
        const int tap = 2 * st + q / 2;
        if (r >= cout || tap > 8) continue;
        const int o = rowmap(r);
        const float inv = 1.0f / (*wscale)[r];
        put_fragment(&frag[(((size_t)st * obtot + ob) * 64 + lane) * 32], DT_F8, 32 * (q % 2),
                     [&](int c) { return w[((size_t)o * cin + c) * 9 + tap] * inv; });
      }
  for (int r = 0; r < cout; ++r) bias[r] = b[rowmap(r)];
  out->cin = cin;
  out->cout = cout;
  out->obtot = obtot;
  out->tc = DT_F8;
  HIP_TRY(dev_malloc((void**)&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  HIP_TRY(dev_alloc(&out->bias, bias.size()));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

// A-operand fragments of the deformable conv (C out, 2C in, G offset groups), in the
// phase order its kernel reduces in.  The 2C input channels are cut into chunks of
// CW = min(CPG, KG) channels (CPG = 2C / G); phase ph covers chunks u = ph*GP + gi,
// gi < GP = KG / CW, each with all nine taps, and is 9 steps of KG deep:
//   frag[((ph*9 + st) * obtot + ob) * 64 + lane] = W[o = 16*ob + lane%16][ci][tap]
// for k = KG*st + (KG/4)*(lane/16) + e, gi = k / (9*CW), tap = (k / CW) % 9,
// ci = (ph*GP + gi)*CW + k % CW.  FP8 fragments are 32 bytes (KG = 128) and hold
// W / s_w[o] with s_w the per output channel scale returned in wscale.
nv_status pack_dcn(nv_context* ctx, const float* w, const float* b, int C, int G, int tc, PackedConv* out,
                   std::vector<float>* wscale) {
  const int KG = tc == DT_F32 ? 16 : (tc == DT_F8 ? 128 : 32);
  const int fb = tc == DT_F8 ? 32 : 16;    // fragment bytes per lane
  const int cin = 2 * C, cpg = cin / G;
  const int CW = cpg < KG ? cpg : KG, GP = KG / CW;
  const int nphase = cin / (GP * CW);
  const int obtot = C / 16;
  std::vector<float> sc((size_t)obtot * 16, 1.0f);
  if (tc == DT_F8) {
    sc = f8_row_scales(w, C, cin, obtot, [](int r) { return r; });
    *wscale = sc;
  }
  std::vector<uint8_t> frag((size_t)nphase * 9 * obtot * 64 * fb, 0);
  for (int ph = 0; ph < nphase; ++ph)
    for (int st = 0; st < 9; ++st)
      for (int ob = 0; ob < obtot; ++ob)
        for (int lane = 0; lane < 64; ++lane) {
          const int o = 16 * ob + lane % 16;
          const int k0 = KG * st + (KG / 4) * (lane / 16);
          const float inv = 1.0f / sc[o];
          put_fragment(&frag[((((size_t)ph * 9 + st) * obtot + ob) * 64 + lane) * fb], tc, 0, [&](int e) {
            const int k = k0 + e;
            const int gi = k / (9 * CW), tap = (k / CW) % 9;
            const int ci = (ph * GP + gi) * CW + k % CW;
            const float v = w[((size_t)o * cin + ci) * 9 + tap];
            return tc == DT_F8 ? v * inv : v;
          });
        }
  out->cin = cin;
  out->cout = C;
  out->obtot = obtot;
  out->tc = tc;
  HIP_TRY(dev_malloc((void**)&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  HIP_TRY(dev_alloc(&out->bias, C));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, b, (size_t)C * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

// Tap-response matrix of the C -> 3 HR conv: row r = 3*tap + o (27 rows, padded to 32),
//   frag[(kg*2 + ob)*64 + lane] = Wr[r = 16*ob + lane%16][c = KG*kg + (KG/4)*(lane/16) + e]
// with Wr[3*tap + o][c] = w[o][c][tap].
nv_status pack_hr(nv_context* ctx, const float* w, const float* b, int cin, int tc, PackedConv* out) {
  const int KG = tc == DT_F32 ? 16 : 32;
  const int nkg = cin / KG;
  std::vector<uint8_t> frag((size_t)nkg * 2 * 64 * 16, 0);
  for (int kg = 0; kg < nkg; ++kg)
    for (int ob = 0; ob < 2; ++ob)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = 16 * ob + lane % 16;
        if (r >= 27) continue;
        const int tap = r / 3, o = r % 3;
        const int c0 = KG * kg + (KG / 4) * (lane / 16);
        put_fragment(&frag[(((size_t)kg * 2 + ob) * 64 + lane) * 16], tc, c0,
                     [&](int c) { return w[((size_t)o * cin + c) * 9 + tap]; });
      }
  std::vector<float> bias(16, 0.0f);
  for (int o = 0; o < 3; ++o) bias[o] = b[o];
  out->cin = cin;
  out->cout = 3;
  out->obtot = 2;
  out->tc = tc;
  HIP_TRY(dev_malloc((void**)&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  HIP_TRY(dev_alloc(&out->bias, bias.size()));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

nv_status upload(nv_context* ctx, const std::vector<float>& v, float** out) {
  HIP_TRY(dev_alloc(out, v.size()));
  ctx->allocs.push_back(*out);
  HIP_TRY(hipMemcpy(*out, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

// Device scales of the FP8 layers (residual convs in order, dcn, up): per-row weight
// scales, output scales and reciprocal activation scales, with every running input
// maximum at zero (activation scale 1) until calibration.
nv_status init_fp8_state(nv_context* ctx, const std::vector<std::vector<float>>& wscales) {
  for (auto& b : ctx->blocks) ctx->q_layers.push_back(&b);
  if (ctx->ut == DT_F8) {
    ctx->q_layers.push_back(&ctx->dcn);
    ctx->q_layers.push_back(&ctx->up);
  }
  if (wscales.size() != ctx->q_layers.size()) return fail(NV_E_INVALID, "FP8 layer count mismatch");
  const size_t nq = ctx->q_layers.size();
  HIP_TRY(dev_alloc(&ctx->q_amax, nq));
  ctx->allocs.push_back(ctx->q_amax);
  HIP_TRY(hipMemset(ctx->q_amax, 0, nq * sizeof(uint32_t)));
  for (size_t l = 0; l < nq; ++l) {
    PackedConv* P = ctx->q_layers[l];
    float* ws = nullptr;
    const nv_status st = upload(ctx, wscales[l], &ws);
    if (st != NV_OK) return st;
    ctx->q_wscale.push_back(ws);
    HIP_TRY(dev_alloc(&P->oscale, (size_t)P->obtot * 16));
    ctx->allocs.push_back(P->oscale);
    HIP_TRY(dev_alloc(&P->ainv, 1));
    ctx->allocs.push_back(P->ainv);
    HIP_TRY(launch_qscale(ctx->q_amax + l, ws, P->oscale, P->ainv, P->obtot * 16, nullptr));
  }
  HIP_TRY(hipDeviceSynchronize());
  return NV_OK;
}

void free_raw(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_workspace(Workspace& ws) {
  free_raw(ws.t0);
  dev_free(ws.o1);
  dev_free(ws.offs);
  free_raw(ws.fmid);
  dev_free(ws.offs_lv);
  free_raw(ws.fmid_lv);
  free_raw(ws.u2);
  dev_free(ws.hr2);
  free_raw(ws.u);
  dev_free(ws.hr);
  for (int i = 0; i < 2; ++i) {
    dev_free(ws.rgb[i]);
    free_raw(ws.feat[i]);
  }
  ws.hp = ws.wp = 0;
  ws.bytes = 0;
}

// Grows the workspace to (hp, wp).  Freeing memory that queued work may still read
// requires the device to be idle first.  The new buffers are allocated into a local
// Workspace and installed only when every allocation succeeded, so a failed growth
// leaves an empty workspace (the next call allocates again), never a partial one.
nv_status ensure_workspace(nv_context* ctx, int hp, int wp) {
  Workspace& ws = ctx->ws;
  if (ws.hp >= hp && ws.wp >= wp && ws.t0) return NV_OK;
  const int nh = hp > ws.hp ? hp : ws.hp, nw = wp > ws.wp ? wp : ws.wp;
  if (ws.t0) {
    HIP_TRY(hipDeviceSynchronize());
    free_workspace(ws);
  }
  const size_t px = (size_t)nh * nw, C = ctx->C, fb = dtype_bytes(ctx->ft);
  Workspace n;
  hipError_t e = dev_malloc(&n.t0, px * C * fb);
  if (e == hipSuccess) e = dev_alloc(&n.o1, px * C);
  if (e == hipSuccess) e = dev_alloc(&n.offs, px * ctx->ldo);
  if (e == hipSuccess) e = dev_malloc(&n.fmid, px * C * fb);
  const size_t r2 = (size_t)ctx->sv * ctx->sh;
  if (e == hipSuccess) e = dev_malloc(&n.u, r2 * px * C * fb);
  if (e == hipSuccess) e = dev_alloc(&n.hr, 3 * r2 * px);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = dev_alloc(&n.rgb[i], 3 * px);
    if (e == hipSuccess) e = dev_malloc(&n.feat[i], feat_bytes(ctx, nh, nw));
  }
  const size_t up = upper_levels_px(ctx, nh, nw);
  if (e == hipSuccess && up) e = dev_alloc(&n.offs_lv, up * ctx->ldo);
  if (e == hipSuccess && up) e = dev_malloc(&n.fmid_lv, up * C * fb);
  if (e == hipSuccess && ctx->side) e = dev_malloc(&n.u2, r2 * px * C * fb);
  if (e == hipSuccess && ctx->side) e = dev_alloc(&n.hr2, 3 * r2 * px);
  if (e != hipSuccess) {
    free_workspace(n);
    return fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "workspace of %dx%d: %s", nw, nh,
                hipGetErrorString(e));
  }
  n.hp = nh;
  n.wp = nw;
  n.bytes = px * (C * fb * (2 + r2) + 4 * C + 4 * (size_t)ctx->ldo + 12 * r2 + 24) +
            2 * feat_bytes(ctx, nh, nw) + up * (4 * (size_t)ctx->ldo + C * fb) +
            (ctx->side ? px * r2 * (C * fb + 12) : 0);
  ws = n;
  return NV_OK;
}

nv_status check_launch(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(NV_E_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return NV_OK;
}

// Runs one launch; with profiling on, brackets it with events on its stream.
template <class F>
nv_status timed(nv_context* ctx, int kind, hipStream_t s, const char* what, F&& launch) {
  hipEvent_t a = nullptr;
  if (ctx && ctx->prof.on && (a = ctx->prof.next()) != nullptr) (void)hipEventRecord(a, s);
  const hipError_t e = launch();
  if (a) {
    hipEvent_t b = ctx->prof.next();
    if (b) {
      (void)hipEventRecord(b, s);
      ctx->prof.recs.push_back({kind, a, b});
    }
  }
  return check_launch(e, what);
}

#define NV_TRY(expr)            \
  do {                          \
    nv_status s_ = (expr);      \
    if (s_ != NV_OK) return s_; \
  } while (0)

nv_status order_begin(Order& o, hipStream_t s) {
  if (o.any && o.last != s) HIP_TRY(hipStreamWaitEvent(s, o.ev, 0));
  return NV_OK;
}

nv_status order_end(Order& o, hipStream_t s) {
  if (!o.ev) HIP_TRY(hipEventCreateWithFlags(&o.ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(o.ev, s));
  o.last = s;
  o.any = true;
  return NV_OK;
}

void order_free(Order& o) {
  if (o.ev) (void)hipEventDestroy(o.ev);
  o = Order{};
}

// Runs body() on HIP stream s after the last users of the buffers behind `ords`, and
// marks s as their last user afterwards (also when body fails part way, since some of
// its work may be queued).
template <class F>
nv_status ordered(std::initializer_list<Order*> ords, hipStream_t s, F&& body) {
  for (Order* o : ords) NV_TRY(order_begin(*o, s));
  const nv_status st = body();
  for (Order* o : ords) {
    const nv_status se = order_end(*o, s);
    if (st == NV_OK && se != NV_OK) return se;
  }
  return st;
}

ConvImg conv_img(const void* src0, const void* src1, const uint32_t* sel, const void* alt0,
                 const void* alt1, const void* res, void* dst, int H, int W) {
  ConvImg im;
  im.src0 = src0;
  im.src1 = src1;
  im.sel = sel;
  im.alt0 = alt0;
  im.alt1 = alt1;
  im.res = res;
  im.dst = dst;
  im.H = H;
  im.W = W;
  im.item_begin = 0;
  return im;
}

// FP8 calibration step of quantised layer l: fold max |x| of its inputs (float16 maps
// of n elements each) into the layer's running maximum, then refresh its scales.
nv_status calib_layer(nv_context* ctx, int l, std::initializer_list<const void*> inputs, size_t n, hipStream_t s) {
  for (const void* x : inputs) NV_TRY(check_launch(launch_amax(DT_F16, x, n, ctx->q_amax + l, s), "amax"));
  PackedConv* P = ctx->q_layers[l];
  return check_launch(launch_qscale(ctx->q_amax + l, ctx->q_wscale[l], P->oscale, P->ainv, P->obtot * 16, s),
                      "qscale");
}

// Whether the residual blocks run as one launch each: 16-bit maps with 64 channels and
// the tuner's choice; FP8 blocks and calibration passes use the separate convs.
static bool resblocks_fused(const nv_context* ctx) {
  return ctx->tune.fused && !ctx->calibrating && !ctx->blocks.empty() &&
         resblock_supported(ctx->blocks[0], ctx->blocks[1], ctx->ft);
}

// The extract stage of one frame in workspace ws (at least hp x wp).
// Levels 2..L of a frame's feature pyramid from its level 1 (section 3.1, the extract
// stage's output): per level the 2x2 mean pool of the level above (into the workspace
// map t0) and the level's conv + LReLU.
nv_status pyramid_impl(nv_context* ctx, Workspace& ws, void* feat, int hp, int wp, hipStream_t s) {
  const int C = ctx->C, ft = ctx->ft, pb = ctx->tune.pb_block;
  for (int l = 2; l <= ctx->levels; ++l) {
    const int h = hp >> (l - 1), w = wp >> (l - 1);
    const void* above = level_map(static_cast<const void*>(feat), ctx, hp, wp, l - 1);
    void* dst = level_map(feat, ctx, hp, wp, l);
    NV_TRY(timed(ctx, NV_K_POOL, s, "pool", [&] { return launch_pool2(ft, above, ws.t0, h, w, C, s); }));
    const ConvImg im = conv_img(ws.t0, nullptr, nullptr, nullptr, nullptr, nullptr, dst, h, w);
    NV_TRY(timed(ctx, NV_K_CONV_BLOCK, s, "down",
                 [&] { return launch_conv(ctx->down[l - 2], CONV_BULK, EPI_LRELU, ft, pb, im, C, 0, s); }));
  }
  return NV_OK;
}

nv_status extract_impl(nv_context* ctx, Workspace& ws, const float* rgb, int hp, int wp, void* feat, hipStream_t s) {
  const int C = ctx->C, ft = ctx->ft, pb = ctx->tune.pb_block;
  NV_TRY(timed(ctx, NV_K_CONV_IN, s, "conv_in",
               [&] { return launch_conv_in(ctx->conv_in, ft, rgb, feat, hp, wp, s); }));
  const size_t n = (size_t)hp * wp * C;
  if (resblocks_fused(ctx)) {
    // ping-pong between feat and the workspace map; an odd block count ends with a copy
    void* a = feat;
    void* b = ws.t0;
    for (int r = 0; r < ctx->cfg.res_blocks; ++r) {
      const ConvImg im = conv_img(a, nullptr, nullptr, nullptr, nullptr, nullptr, b, hp, wp);
      NV_TRY(timed(ctx, NV_K_RESBLOCK, s, "resblock",
                   [&] { return launch_resblock(ctx->blocks[2 * r], ctx->blocks[2 * r + 1], ft, im, s); }));
      std::swap(a, b);
    }
    if (a != feat) HIP_TRY(hipMemcpyAsync(feat, a, n * dtype_bytes(ft), hipMemcpyDeviceToDevice, s));
    return pyramid_impl(ctx, ws, feat, hp, wp, s);
  }
  const ConvImg ia = conv_img(feat, nullptr, nullptr, nullptr, nullptr, nullptr, ws.t0, hp, wp);
  const ConvImg ib = conv_img(ws.t0, nullptr, nullptr, nullptr, nullptr, feat, feat, hp, wp);
  for (int r = 0; r < ctx->cfg.res_blocks; ++r) {
    if (ctx->calibrating) NV_TRY(calib_layer(ctx, 2 * r, {feat}, n, s));
    NV_TRY(timed(ctx, NV_K_CONV_BLOCK, s, "block.a", [&] {
      return launch_conv(ctx->blocks[2 * r], CONV_BULK, EPI_LRELU, ft, pb, ia, C, 0, s);
    }));
    if (ctx->calibrating) NV_TRY(calib_layer(ctx, 2 * r + 1, {ws.t0}, n, s));
    NV_TRY(timed(ctx, NV_K_CONV_BLOCK, s, "block.b", [&] {
      return launch_conv(ctx->blocks[2 * r + 1], CONV_BULK, EPI_RES, ft, pb, ib, C, 0, s);
    }));
  }
  return pyramid_impl(ctx, ws, feat, hp, wp, s);
}

// The fusion stage of group [a, b] in workspace ws (at least hp x wp).  After HR
// output t has been written to hr_out[t], it is packed into pack_out[t] when given.
nv_status fuse_impl(nv_context* ctx, Workspace& ws, const float* rgb_a, const float* rgb_b, const void* fa,
                    const void* fb, int hp, int wp, const uint32_t* sel, uint32_t mask,
                    float* const hr_out[3], float* offs_out, void* fmid_out,
                    const nv_format* pack_fmt, const nv_planes* const pack_out[3], hipStream_t s) {
  const int C = ctx->C, G = ctx->G, ft = ctx->ft;
  float* offs = offs_out ? offs_out : ws.offs;
  void* fmid = fmid_out ? fmid_out : ws.fmid;
  // The t = 0 output needs only frame a, so with the alignment to compute it runs on the
  // side stream beside it (its own HR buffers), joined before the call returns.
  // output t: the pixel-shuffle conv of its features, the HR conv plus the base, the pack
  auto recon = [&](int t, hipStream_t st, void* ub, float* hrb) -> nv_status {
    const void* g = t == 0 ? fa : (t == 1 ? fmid : fb);
    const void* alt = t == 2 ? fa : nullptr;
    const int tsel = t == 0 ? 0 : (t == 1 ? 2 : 1);
    const ConvImg iu = conv_img(g, nullptr, sel, alt, nullptr, nullptr, ub, hp, wp);
    if (ctx->calibrating && ctx->ut == DT_F8)
      NV_TRY(calib_layer(ctx, 2 * ctx->cfg.res_blocks + 1, {g}, (size_t)hp * wp * C, st));
    // scale 1 in both directions: the conv before the (absent) shuffle is a plain conv
    const int r2 = ctx->sv * ctx->sh;
    NV_TRY(timed(ctx, NV_K_UP, st, "up", [&] {
      return launch_conv(ctx->up, CONV_BULK, r2 > 1 ? EPI_SHUFFLE : EPI_LRELU, ft, ctx->tune.pb_up, iu, r2 * C, 0, st);
    }));
    float* hr = hr_out && hr_out[t] ? hr_out[t] : hrb;
    HrImg hi;
    hi.u = ub;
    hi.rgb_a = rgb_a;
    hi.rgb_b = rgb_b;
    hi.sel = sel;
    hi.dst = hr;
    hi.H = hp;
    hi.W = wp;
    hi.tsel = tsel;
    hi.item_begin = 0;
    hi.sv = ctx->sv;
    hi.sh = ctx->sh;
    NV_TRY(timed(ctx, NV_K_HR, st, "hr", [&] { return launch_hr(ctx->hr, ft, hi, st); }));
    if (pack_fmt && pack_out && pack_out[t]) {
      const FrameOut fo = to_frame_out(pack_fmt, pack_out[t]);
      NV_TRY(timed(ctx, NV_K_PACK, st, "pack", [&] { return launch_pack(fo, hr, ctx->sv * hp, ctx->sh * wp, st); }));
    }
    return NV_OK;
  };
  const bool fork = (mask & 1u) && (mask & 6u) && ws.u2 && ws.hr2 && ctx->side && !ctx->calibrating;
  if (fork) {
    HIP_TRY(hipEventRecord(ctx->fork_ev, s));
    HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
    NV_TRY(recon(0, ctx->side, ws.u2, ws.hr2));
    HIP_TRY(hipEventRecord(ctx->join_ev, ctx->side));
  }
  if (mask & 2u) {
    // alignment, coarsest pyramid level first: level l's offsets add twice the x2
    // resize of level l+1's, and its aligned features the x2 resize of level l+1's
    const int L = ctx->levels;
    const size_t px = (size_t)hp * wp, fbytes = dtype_bytes(ft);
    auto offs_at = [&](int l) { return l == 1 ? offs : ws.offs_lv + (level_px_before(hp, wp, l) - px) * ctx->ldo; };
    auto fmid_at = [&](int l) -> void* {
      return l == 1 ? fmid : static_cast<char*>(ws.fmid_lv) + (level_px_before(hp, wp, l) - px) * C * fbytes;
    };
    for (int l = L; l >= 1; --l) {
      const int h = hp >> (l - 1), w = wp >> (l - 1);
      const void* fa_l = level_map(fa, ctx, hp, wp, l);
      const void* fb_l = level_map(fb, ctx, hp, wp, l);
      const PackedConv& O1 = l == 1 ? ctx->off1 : ctx->lvf[l - 2].off1;
      const PackedConv& O2 = l == 1 ? ctx->off2 : ctx->lvf[l - 2].off2;
      const PackedConv& DC = l == 1 ? ctx->dcn : ctx->lvf[l - 2].dcn;
      float* offs_l = offs_at(l);
      void* fmid_l = fmid_at(l);
      const ConvImg i1 = conv_img(fa_l, fb_l, sel, nullptr, fa_l, nullptr, ws.o1, h, w);
      NV_TRY(timed(ctx, NV_K_OFF1, s, "off1",
                   [&] { return launch_conv(O1, CONV_OFF1, EPI_LRELU, ft, ctx->tune.off1, i1, C, 0, s); }));
      const ConvImg i2 = conv_img(ws.o1, nullptr, nullptr, nullptr, nullptr, nullptr, offs_l, h, w);
      NV_TRY(timed(ctx, NV_K_OFF2, s, "off2", [&] {
        return launch_conv(O2, CONV_OFF2, EPI_OFFSET, DT_F32, ctx->tune.off2, i2, ctx->ldo, 18 * G, s);
      }));
      if (l < L)
        NV_TRY(timed(ctx, NV_K_CASCADE, s, "cascade offsets", [&] {
          return launch_up2_add(DT_F32, offs_l, ctx->ldo, offs_at(l + 1), ctx->ldo, h, w, 18 * G, 2.0f, s);
        }));
      DcnImg di;
      di.fa = fa_l;
      di.fb = fb_l;
      di.sel = sel;
      di.offs = offs_l;
      di.dst = fmid_l;
      di.H = h;
      di.W = w;
      di.item_begin = 0;
      if (ctx->calibrating && ctx->ut == DT_F8)
        NV_TRY(calib_layer(ctx, 2 * ctx->cfg.res_blocks, {fa, fb}, (size_t)hp * wp * C, s));
      NV_TRY(timed(ctx, NV_K_DCN, s, "dcn", [&] { return launch_dcn(DC, ft, ctx->tune.pb_dcn, di, ctx->ldo, G, s); }));
      if (l < L)
        NV_TRY(timed(ctx, NV_K_CASCADE, s, "cascade features",
                     [&] { return launch_up2_add(ft, fmid_l, C, fmid_at(l + 1), C, h, w, C, 1.0f, s); }));
    }
  }
  for (int t = 0; t < 3; ++t)
    if ((mask & (1u << t)) && !(fork && t == 0)) NV_TRY(recon(t, s, ws.u, ws.hr));
  if (fork) HIP_TRY(hipStreamWaitEvent(s, ctx->join_ev, 0));
  return NV_OK;
}

// Output frames are the input format scaled by the task's factors.
nv_format out_format(const nv_context* ctx, const nv_format* f) {
  nv_format o = *f;
  o.width *= ctx->sh;
  o.height *= ctx->sv;
  return o;
}

// Copies a frame's planes (codes unchanged): the pass-through of input frames.
nv_status copy_planes(const nv_format* f, const nv_planes* src, const nv_planes* dst, hipStream_t s) {
  const int bps = f->bits == 8 ? 1 : 2;
  for (int i = 0; i < 3; ++i) {
    const int w = (i == 0 || f->chroma == 444) ? f->width : f->width / 2;
    const int h = (i == 0 || f->chroma == 444) ? f->height : f->height / 2;
    HIP_TRY(hipMemcpy2DAsync(dst->data[i], dst->pitch_bytes[i], src->data[i], src->pitch_bytes[i], (size_t)w * bps, h,
                             hipMemcpyDeviceToDevice, s));
  }
  return NV_OK;
}

}  // namespace

extern "C" size_t nv_weight_count(const nv_net_config* cfg) {
  if (!cfg || cfg->channels <= 0 || cfg->offset_groups <= 0 || cfg->res_blocks < 0) return 0;
  return weight_count(*cfg);
}

extern "C" nv_status nv_context_create(int32_t device, const nv_net_config* cfg,
                                       const float* weights, size_t n_floats, nv_context** out) {
  if (!out) return fail(NV_E_INVALID, "out is NULL");
  *out = nullptr;
  NV_TRY(check_config(cfg));
  if (!weights) return fail(NV_E_INVALID, "weights is NULL");
  const size_t need = weight_count(*cfg);
  if (n_floats != need)
    return fail(NV_E_INVALID, "weight blob has %zu floats, this config needs %zu", n_floats, need);
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(NV_E_INVALID, "device %d of %d", device, ndev);
  HIP_TRY(hipSetDevice(device));
  NV_TRY(scratch_setup(device));
  nv_context* ctx = new (std::nothrow) nv_context;
  if (!ctx) return fail(NV_E_NOMEM, "host allocation failed");
  ctx->device = device;
  ctx->cfg = *cfg;
  ctx->C = cfg->channels;
  ctx->G = cfg->offset_groups;
  ctx->ldo = 16 * ((27 * ctx->G + 15) / 16);
  ctx->sv = scale_v(*cfg);
  ctx->sh = scale_h(*cfg);
  ctx->interp = interpolating(*cfg);
  ctx->dbl = doubling(*cfg);
  if (ctx->interp && ctx->dbl) {   // groups emit t = 0 beside the interpolated frame
    hipError_t e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      nv_context_destroy(ctx);
      return fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "side stream: %s", hipGetErrorString(e));
    }
  }
  ctx->ft = cfg->precision == NV_FP16 || cfg->precision == NV_FP8_E4M3
                ? DT_F16
                : (cfg->precision == NV_BF16 ? DT_BF16 : DT_F32);
  ctx->bt = cfg->precision == NV_FP8_E4M3 ? DT_F8 : ctx->ft;
  ctx->ut = (cfg->flags & NV_FLAG_FP8_FUSION) ? DT_F8 : ctx->ft;
  if (ctx->ut == DT_F8) ctx->tune.pb_dcn = 1;   // the FP8 DCN tile is one row per wave
  // the staged DCN form (the tuner's pick wherever it was timed) is the default tile
  else if (dcn_staged_supported(ctx->ft, ctx->ut, ctx->C, ctx->G)) ctx->tune.pb_dcn = 1 | kDcnStaged;
  std::vector<std::vector<float>> wscales;      // FP8 row scales in calibration order
  std::vector<float> dcn_ws, up_ws;
  const auto specs = layer_specs(*cfg);
  ctx->levels = pyramid_levels(*cfg);
  ctx->lvf.resize(ctx->levels - 1);
  const float* p = weights;
  nv_status st = NV_OK;
  for (size_t i = 0; i < specs.size() && st == NV_OK; ++i) {
    const auto& L = specs[i];
    const float* w = p;
    const float* b = p + (size_t)L.cout * L.cin * 9;
    p = b + L.cout;
    const std::string nm = L.name;
    if (nm == "conv_in") {
      ctx->conv_in.cin = 3;
      ctx->conv_in.cout = L.cout;
      st = upload(ctx, std::vector<float>(w, w + (size_t)L.cout * 27), &ctx->conv_in.w);
      if (st == NV_OK) st = upload(ctx, std::vector<float>(b, b + L.cout), &ctx->conv_in.b);
    } else if (nm == "hr") {
      st = pack_hr(ctx, w, b, L.cin, ctx->ft, &ctx->hr);
    } else if (nm == "dcn") {
      std::vector<float> unused;   // row scales are kept for the FP8 (one-level) network only
      st = L.level == 1 ? pack_dcn(ctx, w, b, L.cout, ctx->G, ctx->ut, &ctx->dcn, &dcn_ws)
                        : pack_dcn(ctx, w, b, L.cout, ctx->G, ctx->ut, &ctx->lvf[L.level - 2].dcn, &unused);
    } else {
      // the offset head stays float-class in every precision: float MFMA in FP32 mode
      // (or on request), two-part float16 weights on float16 MFMA otherwise
      const bool head = nm == "off1" || nm == "off2";
      const bool split = head && ctx->ft != DT_F32 && !(cfg->flags & NV_FLAG_HEAD_FP32);
      const int tc = head ? DT_F32 : (nm == "up" ? ctx->ut : ctx->bt);
      PackedConv pc;
      if (split) {
        st = pack_conv_split(ctx, w, b, L.cout, L.cin, nm == "off2" ? 2 : 1, &pc);
      } else if (tc == DT_F8) {
        std::vector<float> ws;
        st = pack_conv_f8(ctx, w, b, L.cout, L.cin, nm == "up" ? ctx->sv * ctx->sh : 1, &pc, &ws);
        if (nm == "up") up_ws = ws;
        else wscales.push_back(ws);
      } else {
        st = pack_conv(ctx, w, b, L.cout, L.cin, nm == "up" ? ctx->sv * ctx->sh : 1, tc, &pc);
      }
      if (nm == "up") {
        pc.sv = ctx->sv;
        pc.sh = ctx->sh;
      }
      if (nm == "block.a" || nm == "block.b") ctx->blocks.push_back(pc);
      else if (nm == "down") ctx->down.push_back(pc);
      else if (nm == "off1") (L.level == 1 ? ctx->off1 : ctx->lvf[L.level - 2].off1) = pc;
      else if (nm == "off2") (L.level == 1 ? ctx->off2 : ctx->lvf[L.level - 2].off2) = pc;
      else if (nm == "up") ctx->up = pc;
    }
  }
  if (st == NV_OK && ctx->bt == DT_F8) {
    if (ctx->ut == DT_F8) {
      wscales.push_back(dcn_ws);
      wscales.push_back(up_ws);
    }
    st = init_fp8_state(ctx, wscales);
  }
  if (st != NV_OK) {
    const std::string msg = g_err;
    nv_context_destroy(ctx);
    g_err = msg;
    return st;
  }
  *out = ctx;
  return NV_OK;
}

extern "C" nv_status nv_context_destroy(nv_context* ctx) {
  if (!ctx) return NV_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  free_workspace(ctx->ws);
  order_free(ctx->ws_ord);
  batch_release(ctx->batch);
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  delete ctx;
  return NV_OK;
}

extern "C" int32_t nv_feature_elem_bytes(const nv_context* ctx) {
  if (!ctx) return 0;
  return ctx->cfg.precision == NV_FP32 ? 4 : 2;
}

extern "C" size_t nv_feature_bytes(const nv_context* ctx, int32_t hp, int32_t wp) {
  if (!ctx || hp <= 0 || wp <= 0) return 0;
  return feat_bytes(ctx, hp, wp);
}

// ---------------------------------------------------------- pixel stages ----

extern "C" nv_status nv_unpack(const nv_format* fmt, const nv_planes* in, float* d_rgb,
                               int32_t hp, int32_t wp, void* stream) {
  NV_TRY(check_format(fmt, "input"));
  NV_TRY(check_planes(fmt, in, "input"));
  if (!d_rgb) return fail(NV_E_INVALID, "d_rgb is NULL");
  if (hp < fmt->height || wp < fmt->width || hp > kMaxDim || wp > kMaxDim || (wp & 3))
    return fail(NV_E_INVALID, "padded size %dx%d must cover the frame and wp be a multiple of 4", wp, hp);
  if ((reinterpret_cast<uintptr_t>(d_rgb) & 15) != 0) return fail(NV_E_INVALID, "d_rgb must be 16-byte aligned");
  return check_launch(launch_unpack(to_frame(fmt, in), d_rgb, hp, wp, (hipStream_t)stream), "unpack");
}

extern "C" nv_status nv_pack(const nv_format* fmt, const float* d_rgb, int32_t rh, int32_t rw,
                             const nv_planes* out, void* stream) {
  NV_TRY(check_format(fmt, "output"));
  NV_TRY(check_planes(fmt, out, "output"));
  if (!d_rgb) return fail(NV_E_INVALID, "d_rgb is NULL");
  if (rh < fmt->height || rw < fmt->width || rh > 2 * kMaxDim || rw > 2 * kMaxDim || (rw & 3))
    return fail(NV_E_INVALID, "RGB size %dx%d must cover the frame and rw be a multiple of 4", rw, rh);
  if ((reinterpret_cast<uintptr_t>(d_rgb) & 15) != 0) return fail(NV_E_INVALID, "d_rgb must be 16-byte aligned");
  return check_launch(launch_pack(to_frame_out(fmt, out), d_rgb, rh, rw, (hipStream_t)stream), "pack");
}

static SceneRule to_rule(const nv_scene_params* p) {
  SceneRule r{24, 1, 4, 1};
  if (p) r = SceneRule{p->mad_thresh_8bit, p->hist_frac_num, p->hist_frac_den, p->enable};
  return r;
}

static nv_status check_scene_params(const nv_scene_params* p) {
  if (!p) return NV_OK;
  if (p->mad_thresh_8bit < 0 || p->hist_frac_num < 0 || p->hist_frac_den <= 0)
    return fail(NV_E_INVALID, "scene thresholds must be non-negative with a positive denominator");
  return NV_OK;
}

extern "C" nv_status nv_scene_metric(const nv_format* fmt, const nv_planes* prev,
                                     const nv_planes* cur, const uint32_t* d_hist_prev,
                                     const nv_scene_params* params, int32_t external_cut,
                                     uint64_t* d_sad, uint32_t* d_hist, uint32_t* d_hd,
                                     uint32_t* d_cut, void* stream) {
  NV_TRY(check_format(fmt, "frame"));
  NV_TRY(check_planes(fmt, cur, "current"));
  if (prev) NV_TRY(check_planes(fmt, prev, "previous"));
  NV_TRY(check_scene_params(params));
  if (external_cut < -1 || external_cut > 1) return fail(NV_E_INVALID, "external_cut must be -1, 0 or 1");
  if (!d_sad || !d_hist || !d_hd || !d_cut) return fail(NV_E_INVALID, "output pointers must be set");
  if (reinterpret_cast<uintptr_t>(d_sad) & 7) return fail(NV_E_INVALID, "d_sad must be 8-byte aligned");
  SceneJob J{};
  J.cur = to_frame(fmt, cur);
  J.prev_y = prev ? prev->data[0] : nullptr;
  J.prev_pitch = prev ? prev->pitch_bytes[0] : 0;
  J.hist_prev = d_hist_prev;
  J.sad = d_sad;
  J.hist = d_hist;
  J.hd = d_hd;
  J.cut = d_cut;
  J.rule = to_rule(params);
  J.external = external_cut;
  return check_launch(launch_scene(J, true, (hipStream_t)stream), "scene");
}

// --------------------------------------------------------------- network ----

static nv_status check_ready(const nv_context* ctx) {
  if (ctx->bt == DT_F8 && !ctx->q_ready)
    return fail(NV_E_INVALID, "FP8 context has no activation scales yet (nv_calibrate or nv_fp8_scales)");
  return NV_OK;
}

// The network of a context was trained for one colourspace; frames of another matrix or
// range are refused (the caller selects the context whose network matches the clip).
static nv_status check_colourspace(const nv_context* ctx, const nv_format* f) {
  if (f->matrix != ctx->cfg.matrix || f->range != ctx->cfg.range)
    return fail(NV_E_UNSUPPORTED, "the network was trained for BT.%d %s range, the frames are BT.%d %s range",
                matrix_number(ctx->cfg.matrix), ctx->cfg.range == NV_RANGE_FULL ? "full" : "limited",
                matrix_number(f->matrix), f->range == NV_RANGE_FULL ? "full" : "limited");
  return NV_OK;
}

static nv_status check_dims(int hp, int wp) {
  if (hp <= 0 || wp <= 0 || hp % 8 || wp % 8 || hp > kMaxDim || wp > kMaxDim)
    return fail(NV_E_INVALID, "padded size %dx%d must be positive multiples of 8", wp, hp);
  return NV_OK;
}

extern "C" nv_status nv_extract(nv_context* ctx, const float* d_rgb, int32_t hp, int32_t wp,
                                void* d_feat, void* stream) {
  if (!ctx || !d_rgb || !d_feat) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_dims(hp, wp));
  NV_TRY(check_ready(ctx));
  hipStream_t s = (hipStream_t)stream;
  NV_TRY(ensure_workspace(ctx, hp, wp));
  return ordered({&ctx->ws_ord}, s, [&] { return extract_impl(ctx, ctx->ws, d_rgb, hp, wp, d_feat, s); });
}

extern "C" nv_status nv_fuse(nv_context* ctx, const float* d_rgb_a, const float* d_rgb_b,
                             const void* d_feat_a, const void* d_feat_b, int32_t hp, int32_t wp,
                             const uint32_t* d_sel, uint32_t out_mask, float* const d_hr[3],
                             float* d_offsets, void* d_fmid, void* stream) {
  if (!ctx || !d_rgb_a || !d_rgb_b || !d_feat_a || !d_feat_b) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_dims(hp, wp));
  if (out_mask == 0 || out_mask > 7) return fail(NV_E_INVALID, "out_mask must be in 1..7");
  if ((out_mask & 2u) && !ctx->interp) return fail(NV_E_INVALID, "t = 1/2 needs an interpolating network");
  NV_TRY(check_ready(ctx));
  for (int t = 0; t < 3; ++t)
    if ((out_mask & (1u << t)) && (!d_hr || !d_hr[t])) return fail(NV_E_INVALID, "d_hr[%d] is NULL", t);
  hipStream_t s = (hipStream_t)stream;
  NV_TRY(ensure_workspace(ctx, hp, wp));
  return ordered({&ctx->ws_ord}, s, [&] {
    return fuse_impl(ctx, ctx->ws, d_rgb_a, d_rgb_b, d_feat_a, d_feat_b, hp, wp, d_sel, out_mask, d_hr, d_offsets,
                     d_fmid, nullptr, nullptr, s);
  });
}

// One group [a, b] in workspace ws: three outputs, t = 0, 1/2, 1.  Without Double frame
// the t = 0 and t = 1 outputs are the input frames passed through unchanged.
static nv_status group_impl(nv_context* ctx, Workspace& ws, const nv_format* fmt, const nv_format* of,
                            const nv_planes in[2], const nv_planes out[3], hipStream_t s) {
  const int hp = round_up(fmt->height, 8), wp = round_up(fmt->width, 8);
  for (int i = 0; i < 2; ++i) {
    const Frame f = to_frame(fmt, &in[i]);
    NV_TRY(timed(ctx, NV_K_UNPACK, s, "unpack", [&] { return launch_unpack(f, ws.rgb[i], hp, wp, s); }));
    NV_TRY(extract_impl(ctx, ws, ws.rgb[i], hp, wp, ws.feat[i], s));
  }
  const nv_planes* po[3] = {&out[0], &out[1], &out[2]};
  if (!ctx->dbl) {
    NV_TRY(copy_planes(fmt, &in[0], &out[0], s));
    NV_TRY(copy_planes(fmt, &in[1], &out[2], s));
  }
  return fuse_impl(ctx, ws, ws.rgb[0], ws.rgb[1], ws.feat[0], ws.feat[1], hp, wp, nullptr, ctx->dbl ? 7u : 2u, nullptr,
                   nullptr, nullptr, of, po, s);
}

static nv_status check_group_task(const nv_context* ctx) {
  if (!ctx->interp)
    return fail(NV_E_UNSUPPORTED, "a network without Interpolation has no frame groups: use a clip stream");
  return NV_OK;
}

extern "C" nv_status nv_enhance_group(nv_context* ctx, const nv_format* fmt, const nv_planes in[2],
                                      const nv_planes out[3], void* stream) {
  if (!ctx || !in || !out) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_ready(ctx));
  NV_TRY(check_group_task(ctx));
  NV_TRY(check_format(fmt, "input"));
  NV_TRY(check_colourspace(ctx, fmt));
  NV_TRY(check_planes(fmt, &in[0], "input 0"));
  NV_TRY(check_planes(fmt, &in[1], "input 1"));
  const nv_format of = out_format(ctx, fmt);
  NV_TRY(check_format(&of, "output"));
  for (int i = 0; i < 3; ++i) NV_TRY(check_planes(&of, &out[i], "output"));
  const int hp = round_up(fmt->height, 8), wp = round_up(fmt->width, 8);
  NV_TRY(ensure_workspace(ctx, hp, wp));
  hipStream_t s = (hipStream_t)stream;
  return ordered({&ctx->ws_ord}, s, [&] { return group_impl(ctx, ctx->ws, fmt, &of, in, out, s); });
}

// ------------------------------------------------- allocation-free group ----

namespace {

// Bytes the group path needs at padded size hp x wp, and (base not null) the workspace
// carved from base with every buffer 256-byte aligned.  Same buffers as ensure_workspace.
size_t static_layout(const nv_context* ctx, int hp, int wp, char* base, Workspace* out) {
  const size_t px = (size_t)hp * wp, C = ctx->C, fb = dtype_bytes(ctx->ft);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  Workspace w;
  w.t0 = take(px * C * fb);
  w.o1 = reinterpret_cast<float*>(take(px * C * 4));
  w.offs = reinterpret_cast<float*>(take(px * ctx->ldo * 4));
  w.fmid = take(px * C * fb);
  const size_t r2 = (size_t)ctx->sv * ctx->sh;
  w.u = take(r2 * px * C * fb);
  w.hr = reinterpret_cast<float*>(take(12 * r2 * px));
  for (int i = 0; i < 2; ++i) {
    w.rgb[i] = reinterpret_cast<float*>(take(12 * px));
    w.feat[i] = take(feat_bytes(ctx, hp, wp));
  }
  const size_t up = upper_levels_px(ctx, hp, wp);
  if (up) {
    w.offs_lv = reinterpret_cast<float*>(take(up * ctx->ldo * 4));
    w.fmid_lv = take(up * C * fb);
  }
  w.hp = hp;
  w.wp = wp;
  w.bytes = off;
  if (out) *out = w;
  return off;
}

}  // namespace

extern "C" nv_status nv_enhance_group_static(nv_context* ctx, const nv_format* fmt, const nv_planes in[2],
                                             const nv_planes out[3], void* stream) {
  if (!ctx || !in || !out) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_ready(ctx));
  NV_TRY(check_group_task(ctx));
  NV_TRY(check_format(fmt, "input"));
  NV_TRY(check_colourspace(ctx, fmt));
  NV_TRY(check_planes(fmt, &in[0], "input 0"));
  NV_TRY(check_planes(fmt, &in[1], "input 1"));
  const nv_format of = out_format(ctx, fmt);
  NV_TRY(check_format(&of, "output"));
  for (int i = 0; i < 3; ++i) NV_TRY(check_planes(&of, &out[i], "output"));
  const int hp = round_up(fmt->height, 8), wp = round_up(fmt->width, 8);
  const size_t need = static_layout(ctx, hp, wp, nullptr, nullptr);
  if (need > (size_t)NV_STATIC_SCRATCH_BYTES)
    return fail(NV_E_INVALID, "a %dx%d group needs %zu bytes of scratch; the static scratch holds %zu",
                fmt->width, fmt->height, need, (size_t)NV_STATIC_SCRATCH_BYTES);
  void* base = scratch_addr(ctx->device);
  if (!base) return fail(NV_E_DEVICE, "static scratch of device %d was not set up", ctx->device);
  Workspace ws;
  static_layout(ctx, hp, wp, static_cast<char*>(base), &ws);
  hipStream_t s = (hipStream_t)stream;
  // launch timing would create events: this entry point runs untimed
  const bool prof = ctx->prof.on;
  ctx->prof.on = false;
  const nv_status st = group_impl(ctx, ws, fmt, &of, in, out, s);
  ctx->prof.on = prof;
  return st;
}

// ------------------------------------------------------------------- FP8 ----

extern "C" nv_status nv_calibrate(nv_context* ctx, const nv_format* fmt, const nv_planes* frames,
                                  int32_t n_frames, void* stream) {
  if (!ctx || !frames) return fail(NV_E_INVALID, "NULL argument");
  if (ctx->bt != DT_F8) return fail(NV_E_INVALID, "only FP8 contexts are calibrated");
  if (n_frames < 2) return fail(NV_E_INVALID, "calibration needs at least 2 frames (got %d)", n_frames);
  NV_TRY(check_format(fmt, "input"));
  NV_TRY(check_colourspace(ctx, fmt));
  for (int i = 0; i < n_frames; ++i) NV_TRY(check_planes(fmt, &frames[i], "calibration frame"));
  const int hp = round_up(fmt->height, 8), wp = round_up(fmt->width, 8);
  NV_TRY(ensure_workspace(ctx, hp, wp));
  hipStream_t s = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  ctx->calibrating = true;
  const nv_status st = ordered({&ctx->ws_ord}, s, [&] {
    HIP_TRY(hipMemsetAsync(ctx->q_amax, 0, ctx->q_layers.size() * sizeof(uint32_t), s));
    nv_status r = NV_OK;
    for (int i = 0; i < n_frames && r == NV_OK; ++i) {
      const int cur = i & 1, prv = cur ^ 1;
      const Frame f = to_frame(fmt, &frames[i]);
      r = check_launch(launch_unpack(f, ws.rgb[cur], hp, wp, s), "unpack");
      if (r == NV_OK) r = extract_impl(ctx, ws, ws.rgb[cur], hp, wp, ws.feat[cur], s);
      if (r == NV_OK && i > 0 && ctx->ut == DT_F8)
        r = fuse_impl(ctx, ws, ws.rgb[prv], ws.rgb[cur], ws.feat[prv], ws.feat[cur], hp, wp, nullptr, 7u, nullptr,
                      nullptr, nullptr, nullptr, nullptr, s);
    }
    return r;
  });
  ctx->calibrating = false;
  if (st != NV_OK) return st;
  ctx->q_ready = true;
  return NV_OK;
}

extern "C" nv_status nv_fp8_scales(nv_context* ctx, float* amax, int32_t n, int32_t set, void* stream) {
  if (!ctx || !amax) return fail(NV_E_INVALID, "NULL argument");
  if (ctx->bt != DT_F8) return fail(NV_E_INVALID, "only FP8 contexts have activation scales");
  const int nq = (int)ctx->q_layers.size();
  if (n != nq) return fail(NV_E_INVALID, "this context has %d FP8 layers (got n = %d)", nq, n);
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint32_t> bits(nq);
  if (!set) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(bits.data(), ctx->q_amax, nq * sizeof(uint32_t), hipMemcpyDeviceToHost));
    for (int l = 0; l < nq; ++l) std::memcpy(&amax[l], &bits[l], 4);
    return NV_OK;
  }
  for (int l = 0; l < nq; ++l) {
    if (!std::isfinite(amax[l]) || amax[l] < 0.0f)
      return fail(NV_E_INVALID, "amax[%d] = %g is not a finite non-negative value", l, (double)amax[l]);
    std::memcpy(&bits[l], &amax[l], 4);
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(ctx->q_amax, bits.data(), nq * sizeof(uint32_t), hipMemcpyHostToDevice));
  for (int l = 0; l < nq; ++l) {
    PackedConv* P = ctx->q_layers[l];
    NV_TRY(check_launch(launch_qscale(ctx->q_amax + l, ctx->q_wscale[l], P->oscale, P->ainv, P->obtot * 16, s),
                        "qscale"));
  }
  ctx->q_ready = true;
  return NV_OK;
}

// ---------------------------------------------------------------- streams ----

// Per-stream device state.  Frame t's pixels and features live in ring slot t % R
// (R >= 2; a batch request of k frames needs R >= k + 1 so the previous call's last
// frame survives while the new ones are written).  luma / hist hold the last pushed
// frame's luma plane and histogram in slot *_last; the next frame writes the other.
struct SceneAcc {
  uint64_t sad;
  uint32_t hist[64];
};

static int64_t luma_pitch(const nv_format* f) { return round_up(f->width * (f->bits == 8 ? 1 : 2), 64); }

struct nv_stream {
  nv_context* ctx = nullptr;
  nv_format fmt{};
  nv_format ofmt{};
  SceneRule rule{};
  int hp = 0, wp = 0;
  int64_t t = 0;                 // frames pushed
  std::vector<float*> rgb;       // R slots [3][hp][wp]
  std::vector<void*> feat;       // R slots [hp][wp][C]
  void* luma[2] = {nullptr, nullptr};
  int luma_last = 0;
  int64_t luma_pitch = 0;
  uint32_t* hist = nullptr;      // [2][64]
  int hist_last = 0;
  uint64_t* sad = nullptr;
  uint32_t* hd = nullptr;
  uint32_t* cuts = nullptr;      // [kCutRing]
  SceneAcc* acc = nullptr;       // scene accumulators, zero between frames
  void* raw[2] = {nullptr, nullptr};   // pass-through task: the last two input frames' planes
  nv_planes raw_planes[2]{};
  Order ord;                     // last call that touched this stream's device state
  size_t bytes = 0;
  int slot(int64_t frame) const { return (int)(frame % (int64_t)rgb.size()); }
};

// Bytes of one frame's planes stored tightly (the pass-through copies).
static size_t raw_frame_bytes(const nv_format* f) {
  const size_t bps = f->bits == 8 ? 1 : 2, luma = (size_t)f->width * f->height;
  return bps * (luma + 2 * (f->chroma == 420 ? luma / 4 : luma));
}

static nv_planes raw_view(const nv_format* f, void* base) {
  nv_planes p;
  const int bps = f->bits == 8 ? 1 : 2;
  const int cw = f->chroma == 420 ? f->width / 2 : f->width, ch = f->chroma == 420 ? f->height / 2 : f->height;
  char* b = static_cast<char*>(base);
  p.data[0] = b;
  p.pitch_bytes[0] = (int64_t)f->width * bps;
  p.data[1] = b + (size_t)f->width * f->height * bps;
  p.pitch_bytes[1] = (int64_t)cw * bps;
  p.data[2] = static_cast<char*>(p.data[1]) + (size_t)cw * ch * bps;
  p.pitch_bytes[2] = (int64_t)cw * bps;
  return p;
}

static size_t slot_bytes(const nv_context* ctx, int hp, int wp) {
  return (size_t)hp * wp * 12 + feat_bytes(ctx, hp, wp);
}

static size_t stream_bytes(const nv_context* ctx, const nv_format* f) {
  const int hp = round_up(f->height, 8), wp = round_up(f->width, 8);
  const size_t raw = ctx->interp && !ctx->dbl ? 2 * raw_frame_bytes(f) : 0;
  return 2 * slot_bytes(ctx, hp, wp) + 2 * (size_t)luma_pitch(f) * f->height + 2 * 64 * 4 + 8 + 4 +
         (size_t)kCutRing * 4 + sizeof(SceneAcc) + raw;
}

static void stream_free(nv_stream* s) {
  for (auto& p : s->rgb) dev_free(p);
  for (auto& p : s->feat) free_raw(p);
  for (int i = 0; i < 2; ++i) free_raw(s->luma[i]);
  dev_free(s->hist);
  dev_free(s->sad);
  dev_free(s->hd);
  dev_free(s->cuts);
  dev_free(s->acc);
  for (int i = 0; i < 2; ++i) free_raw(s->raw[i]);
  order_free(s->ord);
}

// Grows the slot ring to at least r slots, keeping the last pushed frame.
static nv_status stream_ring(nv_stream* s, int r) {
  const int old = (int)s->rgb.size();
  if (old >= r) return NV_OK;
  const size_t px = (size_t)s->hp * s->wp, fbytes = feat_bytes(s->ctx, s->hp, s->wp);
  std::vector<float*> rgb(r, nullptr);
  std::vector<void*> feat(r, nullptr);
  hipError_t e = hipSuccess;
  for (int i = 0; i < r && e == hipSuccess; ++i) {
    e = dev_alloc(&rgb[i], 3 * px);
    if (e == hipSuccess) e = dev_malloc((void**)&feat[i], fbytes);
  }
  if (e == hipSuccess && s->t > 0 && old > 0) {
    HIP_TRY(hipDeviceSynchronize());
    const int from = (int)((s->t - 1) % old), to = (int)((s->t - 1) % r);
    e = hipMemcpy(rgb[to], s->rgb[from], 3 * px * 4, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemcpy(feat[to], s->feat[from], fbytes, hipMemcpyDeviceToDevice);
  }
  if (e != hipSuccess) {
    for (auto& p : rgb) dev_free(p);
    for (auto& p : feat) free_raw(p);
    return fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "stream ring: %s", hipGetErrorString(e));
  }
  if (old > 0) HIP_TRY(hipDeviceSynchronize());
  for (auto& p : s->rgb) dev_free(p);
  for (auto& p : s->feat) free_raw(p);
  s->rgb = rgb;
  s->feat = feat;
  s->bytes += (size_t)(r - old) * slot_bytes(s->ctx, s->hp, s->wp);
  return NV_OK;
}

extern "C" nv_status nv_stream_footprint(const nv_context* ctx, const nv_format* fmt, size_t* bytes) {
  if (!ctx || !bytes) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_format(fmt, "stream"));
  *bytes = stream_bytes(ctx, fmt);
  return NV_OK;
}

extern "C" nv_status nv_stream_open(nv_context* ctx, const nv_format* fmt,
                                    const nv_scene_params* params, nv_stream** out) {
  if (!ctx || !out) return fail(NV_E_INVALID, "NULL argument");
  *out = nullptr;
  NV_TRY(check_format(fmt, "stream"));
  NV_TRY(check_colourspace(ctx, fmt));
  NV_TRY(check_scene_params(params));
  nv_stream* s = new (std::nothrow) nv_stream;
  if (!s) return fail(NV_E_NOMEM, "host allocation failed");
  s->ctx = ctx;
  s->fmt = *fmt;
  s->ofmt = out_format(ctx, fmt);
  s->rule = to_rule(params);
  s->hp = round_up(fmt->height, 8);
  s->wp = round_up(fmt->width, 8);
  s->luma_pitch = luma_pitch(fmt);
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = dev_malloc((void**)&s->luma[i], (size_t)s->luma_pitch * fmt->height);
  if (e == hipSuccess) e = dev_alloc(&s->hist, 128);
  if (e == hipSuccess) e = dev_alloc(&s->sad, 1);
  if (e == hipSuccess) e = dev_alloc(&s->hd, 1);
  if (e == hipSuccess) e = dev_alloc(&s->cuts, kCutRing);
  if (e == hipSuccess) e = dev_alloc(&s->acc, 1);
  if (e == hipSuccess) e = hipMemset(s->acc, 0, sizeof(SceneAcc));
  if (ctx->interp && !ctx->dbl)
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = dev_malloc(&s->raw[i], raw_frame_bytes(fmt));
      if (e == hipSuccess) s->raw_planes[i] = raw_view(fmt, s->raw[i]);
    }
  nv_status st = NV_OK;
  if (e != hipSuccess)
    st = fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "stream allocation: %s", hipGetErrorString(e));
  s->bytes = stream_bytes(ctx, fmt) - 2 * slot_bytes(ctx, s->hp, s->wp);
  if (st == NV_OK) st = stream_ring(s, 2);
  if (st == NV_OK) st = ensure_workspace(ctx, s->hp, s->wp);
  if (st != NV_OK) {
    stream_free(s);
    delete s;
    return st;
  }
  *out = s;
  return NV_OK;
}

// Emits the two outputs of group [a, b]; b's data is used unless *cut_b says frame b
// starts a new scene (then the group is [a, a]).
static nv_status emit_group(nv_stream* s, int slot_a, int slot_b, const uint32_t* cut_b,
                            const nv_planes out[2], hipStream_t hs) {
  const nv_planes* po[3] = {&out[0], &out[1], nullptr};
  NV_TRY(ensure_workspace(s->ctx, s->hp, s->wp));
  if (!s->ctx->dbl) {
    // without Double frame the group's first frame passes through unchanged
    NV_TRY(copy_planes(&s->fmt, &s->raw_planes[slot_a & 1], &out[0], hs));
    return fuse_impl(s->ctx, s->ctx->ws, s->rgb[slot_a], s->rgb[slot_b], s->feat[slot_a], s->feat[slot_b], s->hp,
                     s->wp, cut_b, 2u, nullptr, nullptr, nullptr, &s->ofmt, po, hs);
  }
  return fuse_impl(s->ctx, s->ctx->ws, s->rgb[slot_a], s->rgb[slot_b], s->feat[slot_a], s->feat[slot_b], s->hp,
                   s->wp, cut_b, 3u, nullptr, nullptr, nullptr, &s->ofmt, po, hs);
}

static nv_status push_impl(nv_stream* s, const nv_planes* frame, int32_t external_cut, const nv_planes out[2],
                           int32_t* n_out, hipStream_t hs);

extern "C" nv_status nv_stream_push(nv_stream* s, const nv_planes* frame, int32_t external_cut,
                                    const nv_planes out[2], int32_t* n_out, void* stream) {
  if (!s || !n_out) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_ready(s->ctx));
  NV_TRY(check_planes(&s->fmt, frame, "frame"));
  if (external_cut < -1 || external_cut > 1) return fail(NV_E_INVALID, "external_cut must be -1, 0 or 1");
  if (!s->ctx->interp) {
    if (!out) return fail(NV_E_INVALID, "out is NULL");
    NV_TRY(check_planes(&s->ofmt, &out[0], "output"));
  } else if (s->t > 0) {
    if (!out) return fail(NV_E_INVALID, "out is NULL");
    for (int i = 0; i < 2; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  }
  hipStream_t hs = (hipStream_t)stream;
  return ordered({&s->ctx->ws_ord, &s->ord}, hs, [&] { return push_impl(s, frame, external_cut, out, n_out, hs); });
}

// The scene metric of frame s->t against the previous frame: writes its cut flag at
// *cut_out (device) and keeps its luma plane and histogram for the next frame.
static nv_status scene_step(nv_stream* s, const Frame& f, int32_t external_cut, hipStream_t hs, uint32_t** cut_out) {
  uint32_t* cut_t = s->cuts + (s->t % kCutRing);
  SceneJob J{};
  J.cur = f;
  J.prev_y = s->t > 0 ? s->luma[s->luma_last] : nullptr;
  J.prev_pitch = s->luma_pitch;
  J.hist_prev = s->t > 0 ? s->hist + 64 * s->hist_last : nullptr;
  J.sad = &s->acc->sad;
  J.hist = s->acc->hist;
  J.reset = 1;
  J.hd = s->hd;
  J.cut = cut_t;
  J.hist_save = s->hist + 64 * (s->hist_last ^ 1);
  J.sad_save = s->sad;
  J.luma_save = s->luma[s->luma_last ^ 1];
  J.luma_save_pitch = s->luma_pitch;
  J.rule = s->rule;
  J.external = external_cut;
  NV_TRY(timed(s->ctx, NV_K_SCENE, hs, "scene", [&] { return launch_scene(J, false, hs); }));
  *cut_out = cut_t;
  return NV_OK;
}

// After a frame: the scene state's "previous frame" becomes this one.
static void scene_advance(nv_stream* s) {
  s->t += 1;
  s->luma_last ^= 1;
  s->hist_last ^= 1;
}

// Unpack and extract one frame into ring slot `slot`.
static nv_status frame_in(nv_stream* s, const Frame& f, int slot, hipStream_t hs) {
  NV_TRY(timed(s->ctx, NV_K_UNPACK, hs, "unpack", [&] { return launch_unpack(f, s->rgb[slot], s->hp, s->wp, hs); }));
  NV_TRY(ensure_workspace(s->ctx, s->hp, s->wp));
  return extract_impl(s->ctx, s->ctx->ws, s->rgb[slot], s->hp, s->wp, s->feat[slot], hs);
}

static nv_status push_impl(nv_stream* s, const nv_planes* frame, int32_t external_cut, const nv_planes out[2],
                           int32_t* n_out, hipStream_t hs) {
  const int cur = s->slot(s->t), prv = s->t > 0 ? s->slot(s->t - 1) : 0;
  const Frame f = to_frame(&s->fmt, frame);
  NV_TRY(timed(s->ctx, NV_K_UNPACK, hs, "unpack", [&] { return launch_unpack(f, s->rgb[cur], s->hp, s->wp, hs); }));
  uint32_t* cut_t = nullptr;
  NV_TRY(scene_step(s, f, external_cut, hs, &cut_t));
  NV_TRY(ensure_workspace(s->ctx, s->hp, s->wp));
  NV_TRY(extract_impl(s->ctx, s->ctx->ws, s->rgb[cur], s->hp, s->wp, s->feat[cur], hs));
  *n_out = 0;
  if (!s->ctx->interp) {
    // each frame enhanced alone: one output per input frame, at once
    const nv_planes* po[3] = {&out[0], nullptr, nullptr};
    NV_TRY(fuse_impl(s->ctx, s->ctx->ws, s->rgb[cur], s->rgb[cur], s->feat[cur], s->feat[cur], s->hp, s->wp, nullptr,
                     1u, nullptr, nullptr, nullptr, &s->ofmt, po, hs));
    *n_out = 1;
    scene_advance(s);
    return NV_OK;
  }
  if (!s->ctx->dbl) NV_TRY(copy_planes(&s->fmt, frame, &s->raw_planes[cur & 1], hs));
  if (s->t > 0) {
    NV_TRY(emit_group(s, prv, cur, cut_t, out, hs));
    *n_out = 2;
  }
  scene_advance(s);
  return NV_OK;
}

extern "C" nv_status nv_stream_end(nv_stream* s, const nv_planes out[2], int32_t* n_out, void* stream) {
  if (!s || !n_out) return fail(NV_E_INVALID, "NULL argument");
  *n_out = 0;
  if (s->t == 0 || !s->ctx->interp) return NV_OK;
  if (!out) return fail(NV_E_INVALID, "out is NULL");
  for (int i = 0; i < 2; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  const int last = s->slot(s->t - 1);
  hipStream_t hs = (hipStream_t)stream;
  NV_TRY(ordered({&s->ctx->ws_ord, &s->ord}, hs, [&] { return emit_group(s, last, last, nullptr, out, hs); }));
  *n_out = 2;
  return NV_OK;
}

extern "C" nv_status nv_stream_cuts(nv_stream* s, uint32_t* host_cuts, int32_t n, void* stream) {
  if (!s || (!host_cuts && n > 0)) return fail(NV_E_INVALID, "NULL argument");
  if (n < 0 || n > s->t || n > kCutRing) return fail(NV_E_INVALID, "n = %d but %lld frames pushed", n, (long long)s->t);
  if (n == 0) return NV_OK;
  NV_TRY(order_begin(s->ord, (hipStream_t)stream));
  HIP_TRY(hipMemcpyAsync(host_cuts, s->cuts, (size_t)n * 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  return NV_OK;
}

extern "C" nv_status nv_stream_reset(nv_stream* s) {
  if (!s) return fail(NV_E_INVALID, "NULL argument");
  s->t = 0;
  return NV_OK;
}

extern "C" nv_status nv_stream_close(nv_stream* s) {
  if (!s) return NV_OK;
  (void)hipDeviceSynchronize();
  stream_free(s);
  delete s;
  return NV_OK;
}

// ------------------------------------------ general n, batches of b groups ----
//
// A clip grouped as the paper's framework groups it for a network that consumes n frames
// per run with the Extra frame (n + 1 inputs) and Double frame (2n outputs) flags
// (section 3.1, network integration), run in batches of b groups over the frame store of
// section 3.3 (Fig. 1).  The network here fuses neighbouring frames pairwise, so a
// group's 2n outputs are, for each consumed frame f, HR(f) and the frame between f and
// the group's next input.
//
// Frame store (Fig. 1): P = n b + b positions.  For the block of b groups that starts
// at frame f0 (frames f0 .. f0 + n b), frame f0 + i n (i = 0 .. b: every group's first
// input and the last group's extra input) sits at position b - 1 + i, and frame
// f0 + i n + k (k = 1 .. n - 1) at b - 1 + b + 1 + (k - 1) b + i.  Network input k of
// the b groups is then b consecutive positions, the views of input 0 and of the extra
// input overlap by b - 1 positions, and b n + 1 frames are stored, none twice.  After a
// batch the last frame (f0 + n b) is copied into the chain start (position b - 1) and
// the next block starts there; the first b - 1 positions stay empty.
//
// Grouping (section 3.3): groups never cross a scene cut; the input after a scene's
// last frame is that frame again; a last group short of frames recycles the previous
// group's last frames; a scene shorter than n frames repeats its last frame.  A frame's
// two outputs are emitted once, by the first group that consumes it (a recycled
// group's earlier frames are not computed again).

struct nv_clip {
  nv_stream* st = nullptr;         // scene state; its ring slots are the store positions
  int n = 1, b = 1, P = 0;
  int64_t t = 0;                   // frames pushed
  int64_t scene0 = 0;              // first frame of the current scene
  int64_t f0 = 0;                  // first frame of the current store block
  int64_t next_emit = 0;           // frames before this one have been emitted
  std::vector<int64_t> at;         // frame held at each store position, -1 when none
  std::vector<int32_t> trace;      // see nv_clip_trace
};

namespace {

int clip_pos(const nv_clip* c, int64_t f) {
  const int64_t off = f - c->f0;
  const int base = c->b - 1;
  if (off % c->n == 0) return base + (int)(off / c->n);
  return base + c->b + 1 + (int)((off % c->n) - 1) * c->b + (int)(off / c->n);
}

// The groups of a scene of L frames (scene-relative frame numbers): n + 1 inputs each,
// the first n of them consumed.
std::vector<std::vector<int64_t>> scene_groups(int64_t L, int n) {
  std::vector<int64_t> frames;
  for (int64_t i = 0; i < L; ++i) frames.push_back(i);
  while ((int64_t)frames.size() < n) frames.push_back(L - 1);   // short scene: repeat the last frame
  const int64_t len = (int64_t)frames.size();
  std::vector<std::vector<int64_t>> gs;
  for (int64_t pos = 0; pos < len; pos += n) {
    const int64_t p = pos + n > len ? len - n : pos;             // short last group: recycle
    std::vector<int64_t> in(frames.begin() + p, frames.begin() + p + n);
    in.push_back(p + n < len ? frames[p + n] : L - 1);          // extra input
    gs.push_back(in);
  }
  return gs;
}

// Runs groups (absolute frame numbers, n + 1 inputs each) whose frames are in the store:
// for each consumed frame not yet emitted, its pair with the next input, two outputs.
// Appends the batch to the trace (kind, group count, inputs, store map).
nv_status clip_run(nv_clip* c, int kind, const std::vector<std::vector<int64_t>>& groups, const nv_planes* out,
                   int32_t cap, int32_t* n_out, hipStream_t hs) {
  c->trace.push_back(kind);
  c->trace.push_back((int32_t)groups.size());
  for (const auto& g : groups)
    for (int64_t f : g) c->trace.push_back((int32_t)f);
  for (int64_t f : c->at) c->trace.push_back((int32_t)f);
  for (const auto& g : groups)
    for (int k = 0; k < c->n; ++k) {
      const int64_t f = g[k];
      if (f < c->next_emit) continue;
      if (*n_out + 2 > cap) return fail(NV_E_INVALID, "out has room for %d frames; more are due", cap);
      const int pa = clip_pos(c, f), pb = clip_pos(c, g[k + 1]);
      if (pa < 0 || pa >= c->P || pb < 0 || pb >= c->P || c->at[pa] != f || c->at[pb] != g[k + 1])
        return fail(NV_E_DEVICE, "frame store does not hold frames %lld and %lld", (long long)f,
                    (long long)g[k + 1]);
      NV_TRY(emit_group(c->st, pa, pb, nullptr, out + *n_out, hs));
      *n_out += 2;
      c->next_emit = f + 1;
    }
  return NV_OK;
}

// The groups of the current scene [scene0, end) that the regular batches have not run.
nv_status clip_flush(nv_clip* c, int64_t end, const nv_planes* out, int32_t cap, int32_t* n_out, hipStream_t hs) {
  if (end <= c->scene0) return NV_OK;
  const auto gs = scene_groups(end - c->scene0, c->n);
  const size_t done = (size_t)((c->f0 - c->scene0) / c->n);
  std::vector<std::vector<int64_t>> rest;
  for (size_t i = done; i < gs.size(); ++i) {
    std::vector<int64_t> g = gs[i];
    for (int64_t& f : g) f += c->scene0;
    rest.push_back(g);
  }
  return clip_run(c, 1, rest, out, cap, n_out, hs);
}

}  // namespace

extern "C" nv_status nv_clip_open(nv_context* ctx, const nv_format* fmt, const nv_scene_params* params, int32_t n,
                                  int32_t b, nv_clip** out) {
  if (!ctx || !out) return fail(NV_E_INVALID, "NULL argument");
  *out = nullptr;
  if (n < 1 || b < 1 || n * b + b > kClipMaxPositions)
    return fail(NV_E_INVALID, "n = %d, b = %d: need n, b >= 1 and n b + b <= %d", n, b, kClipMaxPositions);
  if (!ctx->interp || !ctx->dbl)
    return fail(NV_E_UNSUPPORTED, "general-n clips run interpolating networks with Double frame");
  nv_clip* c = new (std::nothrow) nv_clip;
  if (!c) return fail(NV_E_NOMEM, "host allocation failed");
  nv_status st = nv_stream_open(ctx, fmt, params, &c->st);
  c->n = n;
  c->b = b;
  c->P = n * b + b;
  if (st == NV_OK) st = stream_ring(c->st, c->P);
  if (st != NV_OK) {
    if (c->st) nv_stream_close(c->st);
    delete c;
    return st;
  }
  c->at.assign(c->P, -1);
  *out = c;
  return NV_OK;
}

extern "C" nv_status nv_clip_push(nv_clip* c, const nv_planes* frame, int32_t external_cut, const nv_planes* out,
                                  int32_t out_cap, int32_t* n_out, void* stream) {
  if (!c || !n_out) return fail(NV_E_INVALID, "NULL argument");
  *n_out = 0;
  nv_stream* s = c->st;
  NV_TRY(check_ready(s->ctx));
  NV_TRY(check_planes(&s->fmt, frame, "frame"));
  if (external_cut < -1 || external_cut > 1) return fail(NV_E_INVALID, "external_cut must be -1, 0 or 1");
  if (out_cap < 0 || (out_cap > 0 && !out)) return fail(NV_E_INVALID, "out is NULL");
  for (int i = 0; i < out_cap; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  if (c->t >= kCutRing) return fail(NV_E_UNSUPPORTED, "a clip holds at most %d frames", kCutRing);
  hipStream_t hs = (hipStream_t)stream;
  return ordered({&s->ctx->ws_ord, &s->ord}, hs, [&]() -> nv_status {
    const Frame f = to_frame(&s->fmt, frame);
    uint32_t* cut_d = nullptr;
    NV_TRY(scene_step(s, f, external_cut, hs, &cut_d));
    // the grouping depends on where scenes end: the cut flag comes back to the host
    uint32_t cut = 1;
    HIP_TRY(hipMemcpyAsync(&cut, cut_d, sizeof cut, hipMemcpyDeviceToHost, hs));
    HIP_TRY(hipStreamSynchronize(hs));
    const int64_t t = c->t;
    if (t > 0 && cut) {
      NV_TRY(clip_flush(c, t, out, out_cap, n_out, hs));
      c->scene0 = c->f0 = t;
      std::fill(c->at.begin(), c->at.end(), -1);
    }
    const int p = clip_pos(c, t);
    NV_TRY(frame_in(s, f, p, hs));
    c->at[p] = t;
    scene_advance(s);
    c->t = t + 1;
    if (t - c->f0 == (int64_t)c->n * c->b) {
      // a full block: b groups, then the last frame moves to the chain start ("6 to 5")
      std::vector<std::vector<int64_t>> gs;
      for (int g = 0; g < c->b; ++g) {
        std::vector<int64_t> in;
        for (int k = 0; k <= c->n; ++k) in.push_back(c->f0 + (int64_t)g * c->n + k);
        gs.push_back(in);
      }
      NV_TRY(clip_run(c, 0, gs, out, out_cap, n_out, hs));
      const int base = c->b - 1;
      const size_t px = (size_t)s->hp * s->wp;
      HIP_TRY(hipMemcpyAsync(s->rgb[base], s->rgb[p], 12 * px, hipMemcpyDeviceToDevice, hs));
      HIP_TRY(hipMemcpyAsync(s->feat[base], s->feat[p], feat_bytes(s->ctx, s->hp, s->wp), hipMemcpyDeviceToDevice,
                             hs));
      std::fill(c->at.begin(), c->at.end(), -1);
      c->at[base] = t;
      c->f0 = t;
    }
    return NV_OK;
  });
}

extern "C" nv_status nv_clip_end(nv_clip* c, const nv_planes* out, int32_t out_cap, int32_t* n_out, void* stream) {
  if (!c || !n_out) return fail(NV_E_INVALID, "NULL argument");
  *n_out = 0;
  nv_stream* s = c->st;
  if (out_cap < 0 || (out_cap > 0 && !out)) return fail(NV_E_INVALID, "out is NULL");
  for (int i = 0; i < out_cap; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  hipStream_t hs = (hipStream_t)stream;
  return ordered({&s->ctx->ws_ord, &s->ord}, hs, [&] { return clip_flush(c, c->t, out, out_cap, n_out, hs); });
}

extern "C" nv_status nv_clip_trace(const nv_clip* c, int32_t* buf, int32_t cap, int32_t* len) {
  if (!c || !len || (cap > 0 && !buf)) return fail(NV_E_INVALID, "NULL argument");
  *len = (int32_t)c->trace.size();
  for (int32_t i = 0; i < cap && i < *len; ++i) buf[i] = c->trace[i];
  return NV_OK;
}

extern "C" nv_status nv_clip_close(nv_clip* c) {
  if (!c) return NV_OK;
  nv_stream_close(c->st);
  delete c;
  return NV_OK;
}

// ---------------------------------------------------------------- batches ----
//
// A batch runs every stage of many streams' frames and groups as one persistent launch
// per stage over device job tables.  The tables live in a fixed device arena (so the
// recorded graph never changes); each call fills a pinned host copy, uploads it on the
// caller's stream and replays the graph.

namespace {

enum BatchLaunch {
  BL_UNPACK = 0, BL_SCENE, BL_CONV_IN, BL_BLOCK, BL_OFF1, BL_OFF2, BL_DCN, BL_UP, BL_HR, BL_PACK, BL_COUNT
};

struct BatchTables {
  int cnt[BL_COUNT][2];
  UnpackJob unpack[NV_BATCH_MAX_FRAMES];
  SceneJob scene[NV_BATCH_MAX_FRAMES];
  ConvInImg convin[NV_BATCH_MAX_FRAMES];
  ConvImg blk_a[NV_BATCH_MAX_FRAMES];
  ConvImg blk_b[NV_BATCH_MAX_FRAMES];
  ConvImg off1[NV_BATCH_MAX_GROUPS];
  ConvImg off2[NV_BATCH_MAX_GROUPS];
  DcnImg dcn[NV_BATCH_MAX_GROUPS];
  ConvImg up[2][NV_BATCH_MAX_GROUPS];
  HrImg hr[2][NV_BATCH_MAX_GROUPS];
  PackJob pack[2][NV_BATCH_MAX_GROUPS];
};

struct SceneAccum {
  uint64_t sad[NV_BATCH_MAX_FRAMES];
  uint32_t hist[NV_BATCH_MAX_FRAMES][64];
  uint32_t hd[NV_BATCH_MAX_FRAMES];
};

// A growable device buffer carved into per-job pieces (256-byte aligned).
struct Pool {
  char* base = nullptr;
  size_t cap = 0;
};

}  // namespace

struct BatchState {
  BatchTables* host = nullptr;       // pinned staging copy
  BatchTables* dev = nullptr;        // device arena
  SceneAccum* acc = nullptr;         // device scene accumulators
  hipEvent_t uploaded = nullptr;     // staging copy consumed
  hipEvent_t done = nullptr;         // last batch finished with the arena
  bool any = false;
  Pool frame_pool, group_pool;       // per-frame and per-group workspace
  hipStream_t cap = nullptr;         // capture stream
  hipGraphExec_t exec = nullptr;
  bool graph_on = true;
};

namespace {

nv_status pool_reserve(Pool& p, size_t bytes, bool* grew) {
  *grew = false;
  if (bytes <= p.cap) return NV_OK;
  HIP_TRY(hipDeviceSynchronize());
  free_raw(reinterpret_cast<void*&>(p.base));
  p.cap = 0;
  void* b = nullptr;
  HIP_TRY(dev_malloc((void**)&b, bytes));
  p.base = static_cast<char*>(b);
  p.cap = bytes;
  *grew = true;
  return NV_OK;
}

}  // namespace

static void batch_release(BatchState* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->host) (void)hipHostFree(b->host);
  if (b->dev) (void)hipFree(b->dev);
  if (b->acc) (void)hipFree(b->acc);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->done) (void)hipEventDestroy(b->done);
  free_raw(reinterpret_cast<void*&>(b->frame_pool.base));
  free_raw(reinterpret_cast<void*&>(b->group_pool.base));
  delete b;
}

namespace {

// Creates the batch state; it is attached to the context only when every piece of it
// was created, so a failure leaves the context as it was.
nv_status batch_init(nv_context* ctx) {
  if (ctx->batch) return NV_OK;
  BatchState* b = new (std::nothrow) BatchState;
  if (!b) return fail(NV_E_NOMEM, "host allocation failed");
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->host), sizeof(BatchTables), hipHostMallocDefault);
  if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&b->dev), sizeof(BatchTables));
  if (e == hipSuccess) e = dev_malloc(reinterpret_cast<void**>(&b->acc), sizeof(SceneAccum));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    batch_release(b);
    return fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "batch state: %s", hipGetErrorString(e));
  }
  std::memset(b->host, 0, sizeof(BatchTables));
  ctx->batch = b;
  return NV_OK;
}

// Every batched launch of one batch, in dependency order, on stream s.  With timing
// (profiling on, launched directly rather than recorded into the graph) each launch is
// bracketed by the profiler's events.
nv_status batch_enqueue(nv_context* ctx, hipStream_t s, bool timing) {
  BatchTables* T = ctx->batch->dev;
  const int C = ctx->C, G = ctx->G, ft = ctx->ft, pb = ctx->tune.pb_block;
  nv_context* pc = timing ? ctx : nullptr;
  NV_TRY(timed(pc, NV_K_SCENE, s, "scene batch", [&] { return launch_scene_batch(T->scene, T->cnt[BL_SCENE], s); }));
  NV_TRY(timed(pc, NV_K_UNPACK, s, "unpack batch",
               [&] { return launch_unpack_batch(T->unpack, T->cnt[BL_UNPACK], s); }));
  NV_TRY(timed(pc, NV_K_CONV_IN, s, "conv_in batch",
               [&] { return launch_conv_in_batch(ctx->conv_in, ft, T->convin, T->cnt[BL_CONV_IN], s); }));
  for (int r = 0; r < ctx->cfg.res_blocks; ++r) {
    NV_TRY(timed(pc, NV_K_CONV_BLOCK, s, "block.a batch", [&] {
      return launch_conv_batch(ctx->blocks[2 * r], CONV_BULK, EPI_LRELU, ft, pb, T->blk_a, T->cnt[BL_BLOCK], C, 0, s);
    }));
    NV_TRY(timed(pc, NV_K_CONV_BLOCK, s, "block.b batch", [&] {
      return launch_conv_batch(ctx->blocks[2 * r + 1], CONV_BULK, EPI_RES, ft, pb, T->blk_b, T->cnt[BL_BLOCK], C, 0,
                               s);
    }));
  }
  NV_TRY(timed(pc, NV_K_OFF1, s, "off1 batch", [&] {
    return launch_conv_batch(ctx->off1, CONV_OFF1, EPI_LRELU, ft, ctx->tune.off1, T->off1, T->cnt[BL_OFF1], C, 0, s);
  }));
  NV_TRY(timed(pc, NV_K_OFF2, s, "off2 batch", [&] {
    return launch_conv_batch(ctx->off2, CONV_OFF2, EPI_OFFSET, DT_F32, ctx->tune.off2, T->off2, T->cnt[BL_OFF2],
                             ctx->ldo, 18 * G, s);
  }));
  NV_TRY(timed(pc, NV_K_DCN, s, "dcn batch", [&] {
    return launch_dcn_batch(ctx->dcn, ft, ctx->tune.pb_dcn, T->dcn, T->cnt[BL_DCN], ctx->ldo, G, s);
  }));
  for (int o = 0; o < 2; ++o) {
    NV_TRY(timed(pc, NV_K_UP, s, "up batch", [&] {
      return launch_conv_batch(ctx->up, CONV_BULK, EPI_SHUFFLE, ft, ctx->tune.pb_up, T->up[o], T->cnt[BL_UP], 4 * C,
                               0, s);
    }));
    NV_TRY(timed(pc, NV_K_HR, s, "hr batch", [&] { return launch_hr_batch(ctx->hr, ft, T->hr[o], T->cnt[BL_HR], s); }));
    NV_TRY(timed(pc, NV_K_PACK, s, "pack batch", [&] { return launch_pack_batch(T->pack[o], T->cnt[BL_PACK], s); }));
  }
  return NV_OK;
}

struct FrameRef {          // one frame of the batch
  nv_stream* s;
  int64_t t;               // its index in the stream
  const nv_planes* in;
  int ext;
  int first, last;         // first / last frame of its request
};

struct GroupRef {          // one emitted group
  nv_stream* s;
  int slot_a, slot_b;
  const uint32_t* sel;     // cut flag of frame b, or null for [a, a]
  const nv_planes* out;    // two output frames
};

}  // namespace

extern "C" nv_status nv_batch_graph(nv_context* ctx, int32_t on) {
  if (!ctx) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(batch_init(ctx));
  ctx->batch->graph_on = on != 0;
  return NV_OK;
}

extern "C" nv_status nv_batch_bytes_per_px(const nv_context* ctx, size_t* per_group, size_t* per_frame) {
  if (!ctx || !per_group || !per_frame) return fail(NV_E_INVALID, "NULL argument");
  const size_t C = ctx->C, fb = dtype_bytes(ctx->ft);
  // a group's offset-head hidden map, offsets, aligned features, HR features and HR
  // R'G'B'; a frame's features (the batch pools, before 256-byte rounding per buffer)
  *per_group = C * 4 + (size_t)ctx->ldo * 4 + C * fb + 4 * C * fb + 48;
  *per_frame = C * fb;
  return NV_OK;
}

extern "C" nv_status nv_batch_footprint(const nv_context* ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(NV_E_INVALID, "NULL argument");
  *bytes = ctx->batch ? ctx->batch->frame_pool.cap + ctx->batch->group_pool.cap + sizeof(BatchTables) +
                            sizeof(SceneAccum)
                      : 0;
  return NV_OK;
}

extern "C" nv_status nv_enhance_batch(nv_context* ctx, const nv_batch_req* reqs, int32_t n, void* stream) {
  if (!ctx || (!reqs && n > 0) || n < 0) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_ready(ctx));
  if (!default_task(ctx->cfg))
    return fail(NV_E_UNSUPPORTED, "batches run the x2 space-time task; other tasks use clip streams");
  if (ctx->levels > 1)
    return fail(NV_E_UNSUPPORTED, "batches run one-level networks; feature pyramids use clip streams");
  hipStream_t hs = (hipStream_t)stream;
  // ---- validation (nothing is enqueued or changed before it passes) ----
  int nframes = 0, ngroups = 0;
  for (int i = 0; i < n; ++i) {
    const nv_batch_req& r = reqs[i];
    if (!r.stream || r.stream->ctx != ctx) return fail(NV_E_INVALID, "request %d: stream is NULL or of another context", i);
    for (int k = 0; k < i; ++k)
      if (reqs[k].stream == r.stream) return fail(NV_E_INVALID, "requests %d and %d share a stream", k, i);
    if (r.n_frames < 1 || r.n_frames > NV_BATCH_MAX_CHAIN)
      return fail(NV_E_INVALID, "request %d: n_frames must be 1..%d", i, (int)NV_BATCH_MAX_CHAIN);
    if (!r.frames || !r.n_out) return fail(NV_E_INVALID, "request %d: NULL frames or n_out", i);
    const int emitted = r.n_frames - (r.stream->t == 0 ? 1 : 0) + (r.end_of_clip ? 1 : 0);
    if (emitted > 0 && !r.out) return fail(NV_E_INVALID, "request %d: out is NULL", i);
    for (int j = 0; j < r.n_frames; ++j) {
      NV_TRY(check_planes(&r.stream->fmt, &r.frames[j], "batch frame"));
      if (r.external_cut && (r.external_cut[j] < -1 || r.external_cut[j] > 1))
        return fail(NV_E_INVALID, "request %d: external_cut must be -1, 0 or 1", i);
    }
    for (int o = 0; o < 2 * emitted; ++o) NV_TRY(check_planes(&r.stream->ofmt, &r.out[o], "batch output"));
    nframes += r.n_frames;
    ngroups += emitted;
  }
  if (nframes > NV_BATCH_MAX_FRAMES || ngroups > NV_BATCH_MAX_GROUPS)
    return fail(NV_E_INVALID, "batch of %d frames / %d groups exceeds %d / %d", nframes, ngroups,
                (int)NV_BATCH_MAX_FRAMES, (int)NV_BATCH_MAX_GROUPS);
  NV_TRY(batch_init(ctx));
  BatchState* B = ctx->batch;
  for (int i = 0; i < n; ++i) NV_TRY(stream_ring(reqs[i].stream, reqs[i].n_frames + 1));

  // ---- frames and groups in emission order ----
  std::vector<FrameRef> frames;
  std::vector<GroupRef> groups;
  for (int i = 0; i < n; ++i) {
    const nv_batch_req& r = reqs[i];
    nv_stream* s = r.stream;
    int emitted = 0;
    for (int j = 0; j < r.n_frames; ++j) {
      const int64_t t = s->t + j;
      frames.push_back({s, t, &r.frames[j], r.external_cut ? r.external_cut[j] : -1, j == 0, j == r.n_frames - 1});
      if (t > 0) groups.push_back({s, s->slot(t - 1), s->slot(t), s->cuts + (t % kCutRing), &r.out[2 * emitted++]});
    }
    if (r.end_of_clip) {
      const int last = s->slot(s->t + r.n_frames - 1);
      groups.push_back({s, last, last, nullptr, &r.out[2 * emitted++]});
    }
    *r.n_out = 2 * emitted;
  }

  // ---- workspace ----
  const int C = ctx->C, fbytes = dtype_bytes(ctx->ft);
  size_t fneed = 0, gneed = 0;
  for (const auto& f : frames) fneed += align256((size_t)f.s->hp * f.s->wp * C * fbytes);
  for (const auto& g : groups) {
    const size_t px = (size_t)g.s->hp * g.s->wp;
    gneed += align256(px * C * 4) + align256(px * ctx->ldo * 4) + align256(px * C * fbytes) +
             align256(4 * px * C * fbytes) + align256(12 * px * 4);
  }
  bool grew = false;
  NV_TRY(pool_reserve(B->frame_pool, fneed, &grew));
  NV_TRY(pool_reserve(B->group_pool, gneed, &grew));

  // ---- job tables ----
  if (B->any) HIP_TRY(hipEventSynchronize(B->uploaded));   // staging copy free again
  BatchTables& T = *B->host;
  const int pbb = ctx->tune.pb_block, pbu = ctx->tune.pb_up, pbd = ctx->tune.pb_dcn & (kDcnWindow - 1);
  int it[BL_COUNT] = {0};
  char* fp = B->frame_pool.base;
  for (size_t k = 0; k < frames.size(); ++k) {
    const FrameRef& F = frames[k];
    nv_stream* s = F.s;
    const int hp = s->hp, wp = s->wp, sl = s->slot(F.t);
    const Frame fr = to_frame(&s->fmt, F.in);
    UnpackJob& u = T.unpack[k];
    u.f = fr;
    u.m = make_inv(fr.bits, fr.matrix, fr.full);
    u.rgb = s->rgb[sl];
    u.hp = hp;
    u.wp = wp;
    u.item_begin = it[BL_UNPACK];
    it[BL_UNPACK] += unpack_items(hp, wp);
    SceneJob& sc = T.scene[k];
    sc.cur = fr;
    if (F.t == 0) {
      sc.prev_y = nullptr;
      sc.prev_pitch = 0;
      sc.hist_prev = nullptr;
    } else if (F.first) {
      sc.prev_y = s->luma[s->luma_last];
      sc.prev_pitch = s->luma_pitch;
      sc.hist_prev = s->hist + 64 * s->hist_last;
    } else {
      sc.prev_y = frames[k - 1].in->data[0];
      sc.prev_pitch = frames[k - 1].in->pitch_bytes[0];
      sc.hist_prev = B->acc->hist[k - 1];
    }
    sc.sad = &B->acc->sad[k];
    sc.hist = B->acc->hist[k];
    sc.hd = &B->acc->hd[k];
    sc.cut = s->cuts + (F.t % kCutRing);
    sc.hist_save = F.last ? s->hist + 64 * (s->hist_last ^ 1) : nullptr;
    sc.luma_save = F.last ? s->luma[s->luma_last ^ 1] : nullptr;
    sc.luma_save_pitch = s->luma_pitch;
    sc.sad_save = nullptr;
    sc.reset = 0;
    sc.rule = s->rule;
    sc.external = F.ext;
    sc.item_begin = it[BL_SCENE];
    it[BL_SCENE] += scene_items(fr.h);
    void* t0 = fp;
    fp += align256((size_t)hp * wp * C * fbytes);
    ConvInImg& ci = T.convin[k];
    ci.rgb = s->rgb[sl];
    ci.dst = s->feat[sl];
    ci.H = hp;
    ci.W = wp;
    ci.item_begin = it[BL_CONV_IN];
    it[BL_CONV_IN] += conv_in_items(hp, wp, C);
    const int nobg = ctx->blocks.empty() ? 1 : ctx->blocks[0].obtot / conv_ob(CONV_BULK, EPI_LRELU, ctx->blocks[0].obtot, ctx->blocks[0].tc, pbb);
    T.blk_a[k] = conv_img(s->feat[sl], nullptr, nullptr, nullptr, nullptr, nullptr, t0, hp, wp);
    T.blk_b[k] = conv_img(t0, nullptr, nullptr, nullptr, nullptr, s->feat[sl], s->feat[sl], hp, wp);
    T.blk_a[k].item_begin = T.blk_b[k].item_begin = it[BL_BLOCK];
    it[BL_BLOCK] += conv_items(hp, wp, tile_pb(pbb), nobg);
  }
  char* gp = B->group_pool.base;
  for (size_t k = 0; k < groups.size(); ++k) {
    const GroupRef& Gr = groups[k];
    nv_stream* s = Gr.s;
    const int hp = s->hp, wp = s->wp;
    const size_t px = (size_t)hp * wp;
    float* o1 = reinterpret_cast<float*>(gp);
    gp += align256(px * C * 4);
    float* offs = reinterpret_cast<float*>(gp);
    gp += align256(px * ctx->ldo * 4);
    void* fmid = gp;
    gp += align256(px * C * fbytes);
    void* u = gp;
    gp += align256(4 * px * C * fbytes);
    float* hr = reinterpret_cast<float*>(gp);
    gp += align256(12 * px * 4);
    const void* fa = s->feat[Gr.slot_a];
    const void* fb = s->feat[Gr.slot_b];
    const float* ra = s->rgb[Gr.slot_a];
    const float* rb = s->rgb[Gr.slot_b];
    T.off1[k] = conv_img(fa, fb, Gr.sel, nullptr, fa, nullptr, o1, hp, wp);
    T.off1[k].item_begin = it[BL_OFF1];
    it[BL_OFF1] += conv_items(hp, wp, tile_pb(ctx->tune.off1),
                              ctx->off1.obtot / conv_ob(CONV_OFF1, EPI_LRELU, ctx->off1.obtot, ctx->off1.tc, ctx->tune.off1));
    T.off2[k] = conv_img(o1, nullptr, nullptr, nullptr, nullptr, nullptr, offs, hp, wp);
    T.off2[k].item_begin = it[BL_OFF2];
    it[BL_OFF2] += conv_items(hp, wp, tile_pb(ctx->tune.off2),
                              ctx->off2.obtot / conv_ob(CONV_OFF2, EPI_OFFSET, ctx->off2.obtot, ctx->off2.tc, ctx->tune.off2));
    DcnImg& d = T.dcn[k];
    d.fa = fa;
    d.fb = fb;
    d.sel = Gr.sel;
    d.offs = offs;
    d.dst = fmid;
    d.H = hp;
    d.W = wp;
    d.item_begin = it[BL_DCN];
    it[BL_DCN] += conv_items(hp, wp, pbd, 1);
    for (int o = 0; o < 2; ++o) {
      T.up[o][k] = conv_img(o == 0 ? fa : fmid, nullptr, Gr.sel, nullptr, nullptr, nullptr, u, hp, wp);
      T.up[o][k].item_begin = it[BL_UP];
      HrImg& h = T.hr[o][k];
      h.u = u;
      h.rgb_a = ra;
      h.rgb_b = rb;
      h.sel = Gr.sel;
      h.dst = hr;
      h.H = hp;
      h.W = wp;
      h.tsel = o == 0 ? 0 : 2;
      h.item_begin = it[BL_HR];
      h.sv = h.sh = 2;
      PackJob& pk = T.pack[o][k];
      pk.f = to_frame_out(&s->ofmt, &Gr.out[o]);
      pk.m = make_fwd(pk.f.bits, pk.f.matrix, pk.f.full);
      pk.rgb = hr;
      pk.rh = 2 * hp;
      pk.rw = 2 * wp;
      pk.item_begin = it[BL_PACK];
    }
    it[BL_UP] += conv_items(hp, wp, tile_pb(pbu), ctx->up.obtot / conv_ob(CONV_BULK, EPI_SHUFFLE, ctx->up.obtot, ctx->up.tc, pbu));
    it[BL_HR] += hr_items(hp, wp);
    it[BL_PACK] += pack_items(s->ofmt.width, s->ofmt.height, s->ofmt.chroma);
  }
  const int nf = (int)frames.size(), ng = (int)groups.size();
  const int njobs[BL_COUNT] = {nf, nf, nf, nf, ng, ng, ng, ng, ng, ng};
  for (int k = 0; k < BL_COUNT; ++k) {
    T.cnt[k][0] = njobs[k];
    T.cnt[k][1] = njobs[k] > 0 ? it[k] : 0;
  }

  // ---- upload, then launch (graph replay or direct) ----
  if (B->any) HIP_TRY(hipStreamWaitEvent(hs, B->done, 0));
  for (int i = 0; i < n; ++i) NV_TRY(order_begin(reqs[i].stream->ord, hs));
  HIP_TRY(hipMemcpyAsync(B->dev, B->host, sizeof(BatchTables), hipMemcpyHostToDevice, hs));
  HIP_TRY(hipEventRecord(B->uploaded, hs));
  B->any = true;
  if (B->graph_on) {
    if (!B->exec) {
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeRelaxed));
      const nv_status st = batch_enqueue(ctx, B->cap, false);
      const hipError_t ec = hipStreamEndCapture(B->cap, &g);
      if (st != NV_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      HIP_TRY(ec);
      const hipError_t ei = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_TRY(ei);
    }
    HIP_TRY(hipGraphLaunch(B->exec, hs));
  } else {
    NV_TRY(batch_enqueue(ctx, hs, true));
  }
  HIP_TRY(hipEventRecord(B->done, hs));
  for (int i = 0; i < n; ++i) NV_TRY(order_end(reqs[i].stream->ord, hs));

  // ---- stream states advance ----
  for (int i = 0; i < n; ++i) {
    nv_stream* s = reqs[i].stream;
    s->t += reqs[i].n_frames;
    s->luma_last ^= 1;
    s->hist_last ^= 1;
  }
  (void)grew;
  return NV_OK;
}

// --------------------------------------------------------------- autotuner ----

namespace {

std::string tile_name(int code) {
  char b[32];
  if (tile_lw(code)) snprintf(b, sizeof b, "pb%dlw", tile_pb(code));
  else if (tile_m32(code)) snprintf(b, sizeof b, "pb%dm32", tile_pb(code));
  else if (tile_wo(code) == 1) snprintf(b, sizeof b, "pb%d", tile_pb(code));
  else snprintf(b, sizeof b, "pb%dw%d", tile_pb(code), tile_wo(code));
  return b;
}

// The DCN tile codes the tuner times for a network: rows per wave, the windowed forms
// and the staged form where the maps and offset groups allow them.
std::vector<int> dcn_tiles(int ft, int tc, int C, int groups) {
  std::vector<int> v{1, 2};
  if (dcn_window_supported(ft, tc, C, groups)) {
    v.push_back(1 | kDcnWindow);
    v.push_back(2 | kDcnWindow);
  }
  if (dcn_staged_supported(ft, tc, C, groups)) v.push_back(1 | kDcnStaged);
  return v;
}

std::string dcn_tile_name(int code) {
  char b[32];
  snprintf(b, sizeof b, "pb%d%s", code & (kDcnWindow - 1),
           (code & kDcnWindow) ? "win" : (code & kDcnStaged) ? "stg" : "");
  return b;
}

template <class F>
nv_status time_launch(hipStream_t s, int reps, float* ms, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  NV_TRY(check_launch(launch(), "autotune warmup"));
  HIP_TRY(hipEventRecord(a, s));
  for (int r = 0; r < reps; ++r) NV_TRY(check_launch(launch(), "autotune"));
  HIP_TRY(hipEventRecord(b, s));
  HIP_TRY(hipEventSynchronize(b));
  float t = 0.0f;
  HIP_TRY(hipEventElapsedTime(&t, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = t / reps;
  return NV_OK;
}

}  // namespace

extern "C" nv_status nv_autotune(nv_context* ctx, int32_t hp, int32_t wp, void* stream, char* report,
                                 size_t report_len) {
  if (!ctx) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_dims(hp, wp));
  const char* cache = getenv("NNVISR_TUNE_CACHE");
  char key[128];
  snprintf(key, sizeof key, "prec=%d C=%d R=%d size=%dx%d", ctx->cfg.precision, ctx->C, ctx->cfg.res_blocks,
           wp, hp);
  if (!default_task(ctx->cfg)) {   // the task changes the pixel-shuffle conv and drops the alignment
    const size_t n = strlen(key);
    snprintf(key + n, sizeof key - n, " task=%dx%d/%d%d", ctx->sv, ctx->sh, (int)ctx->interp, (int)ctx->dbl);
  }
  std::string rep;
  bool found = false;
  if (cache) {
    if (FILE* f = fopen(cache, "r")) {
      char line[256];
      while (fgets(line, sizeof line, f)) {
        int a = 0, b = 0, c = 0, d = 2, e = 2, fz = 0;
        char k2[128];
        if (sscanf(line, "%127[^|]| %d %d %d %d %d %d", k2, &a, &b, &c, &d, &e, &fz) >= 4) {
          std::string ks(k2);
          while (!ks.empty() && ks.back() == ' ') ks.pop_back();
          if (ks == key && a > 0 && b > 0 && c > 0 && d > 0 && e > 0) {
            ctx->tune.pb_block = a;
            ctx->tune.pb_up = b;
            ctx->tune.pb_dcn = c;
            ctx->tune.off1 = d;
            ctx->tune.off2 = e;
            ctx->tune.fused = fz != 0;
            found = true;
          }
        }
      }
      fclose(f);
    }
  }
  if (!found) {
    NV_TRY(ensure_workspace(ctx, hp, wp));
    hipStream_t s = (hipStream_t)stream;
    NV_TRY(order_begin(ctx->ws_ord, s));
    Workspace& ws = ctx->ws;
    const int C = ctx->C, ft = ctx->ft;
    // inputs for the timing runs: zero offsets keep every DCN sample inside the frame
    HIP_TRY(hipMemsetAsync(ws.feat[0], 0, (size_t)hp * wp * C * dtype_bytes(ft), s));
    HIP_TRY(hipMemsetAsync(ws.offs, 0, (size_t)hp * wp * ctx->ldo * 4, s));
    HIP_TRY(hipMemsetAsync(ws.o1, 0, (size_t)hp * wp * C * 4, s));
    char buf[256];
    // bulk conv tiles: rows per wave 1, 2, 4, and with two waves along the output blocks
    // rows per wave 1, 2 (16-bit / FP8 also 4: the float form would need twice the
    // fragment registers)
    std::vector<int> bulk_tiles = {1, 2, 4};
    for (int pb : {1, 2}) bulk_tiles.push_back(tile_code(pb, 2));
    if (ft != DT_F32) {
      bulk_tiles.push_back(tile_code(4, 2));
      // LDS-resident weights, where the device allows the workgroup that much LDS
      if (C == 64 && lds_weight_tiles())
        for (int pb : {2, 4})
          if (bulk_tile_lds(ctx->bt, C, tile_code(pb, 1, 1)) <= lds_limit() &&
              bulk_tile_lds(ctx->ut, C, tile_code(pb, 1, 1)) <= lds_limit())
            bulk_tiles.push_back(tile_code(pb, 1, 1));
    }
    // split offset head: rows per wave 2 (all output blocks) or 4 (two blocks), or two
    // waves along the output blocks
    auto head_tiles = [&](const PackedConv& P) {
      std::vector<int> t = {tile_code(2, 1)};
      if (P.tc == DT_F16 && P.obtot % 2 == 0) {
        t.push_back(tile_code(4, 1));
        t.push_back(tile_code(2, 2));
      }
      return t;
    };
    // 32x32x16 MFMA form for 16-bit convs with 64 input channels
    std::vector<int> block_tiles = bulk_tiles, up_tiles = bulk_tiles;
    const int r2 = ctx->sv * ctx->sh, up_epi = r2 > 1 ? EPI_SHUFFLE : EPI_LRELU;
    if (C == 64) {
      for (int pb : {2, 4}) {
        if (!ctx->blocks.empty() && ctx->blocks[0].frag32) block_tiles.push_back(tile_code(pb, 1, 0, 1));
        if (ctx->up.frag32) up_tiles.push_back(tile_code(pb, 1, 0, 1));
      }
    }
    struct Cand {
      const char* name;
      int* slot;
      std::vector<int> pbs;
    } cands[5] = {{"block", &ctx->tune.pb_block, block_tiles}, {"up", &ctx->tune.pb_up, up_tiles},
                  {"dcn", &ctx->tune.pb_dcn,
                   ctx->ut == DT_F8 ? std::vector<int>{1}
                   : dcn_tiles(ft, ctx->dcn.tc, C, ctx->G)},
                  {"off1", &ctx->tune.off1, head_tiles(ctx->off1)}, {"off2", &ctx->tune.off2, head_tiles(ctx->off2)}};
    for (auto& cd : cands) {
      // networks that do not interpolate have no offset head and no alignment
      if (!ctx->interp && cd.slot != &ctx->tune.pb_block && cd.slot != &ctx->tune.pb_up) continue;
      float best = 1e30f;
      int best_pb = *cd.slot;
      rep += cd.name;
      rep += ":";
      for (int pb : cd.pbs) {
        float ms = 0.0f;
        nv_status st;
        if (cd.slot == &ctx->tune.pb_block) {
          const ConvImg im = conv_img(ws.feat[0], nullptr, nullptr, nullptr, nullptr, nullptr, ws.t0, hp, wp);
          st = time_launch(s, 3, &ms, [&] {
            return launch_conv(ctx->blocks.empty() ? ctx->up : ctx->blocks[0], CONV_BULK,
                               ctx->blocks.empty() ? up_epi : EPI_LRELU, ft, pb, im,
                               ctx->blocks.empty() ? r2 * C : C, 0, s);
          });
        } else if (cd.slot == &ctx->tune.pb_up) {
          const ConvImg im = conv_img(ws.feat[0], nullptr, nullptr, nullptr, nullptr, nullptr, ws.u, hp, wp);
          st = time_launch(s, 3, &ms, [&] { return launch_conv(ctx->up, CONV_BULK, up_epi, ft, pb, im, r2 * C, 0, s); });
        } else if (cd.slot == &ctx->tune.off1) {
          const ConvImg im = conv_img(ws.feat[0], ws.feat[0], nullptr, nullptr, nullptr, nullptr, ws.o1, hp, wp);
          st = time_launch(s, 3, &ms, [&] { return launch_conv(ctx->off1, CONV_OFF1, EPI_LRELU, ft, pb, im, C, 0, s); });
        } else if (cd.slot == &ctx->tune.off2) {
          const ConvImg im = conv_img(ws.o1, nullptr, nullptr, nullptr, nullptr, nullptr, ws.offs, hp, wp);
          st = time_launch(s, 3, &ms, [&] {
            return launch_conv(ctx->off2, CONV_OFF2, EPI_OFFSET, DT_F32, pb, im, ctx->ldo, 18 * ctx->G, s);
          });
        } else {
          DcnImg di;
          di.fa = ws.feat[0];
          di.fb = ws.feat[0];
          di.sel = nullptr;
          di.offs = ws.offs;
          di.dst = ws.fmid;
          di.H = hp;
          di.W = wp;
          di.item_begin = 0;
          st = time_launch(s, 3, &ms, [&] { return launch_dcn(ctx->dcn, ft, pb, di, ctx->ldo, ctx->G, s); });
        }
        if (st != NV_OK) return st;
        snprintf(buf, sizeof buf, " %s=%.1fus",
                 (cd.slot == &ctx->tune.pb_dcn ? dcn_tile_name(pb) : tile_name(pb)).c_str(), 1000.0f * ms);
        rep += buf;
        if (ms < best) {
          best = ms;
          best_pb = pb;
        }
      }
      *cd.slot = best_pb;
      snprintf(buf, sizeof buf, " -> %s; ",
               (cd.slot == &ctx->tune.pb_dcn ? dcn_tile_name(best_pb) : tile_name(best_pb)).c_str());
      rep += buf;
    }
    // residual block: one fused launch against the two convs with the chosen tile
    if (!ctx->blocks.empty() && resblock_supported(ctx->blocks[0], ctx->blocks[1], ft)) {
      float t_fused = 0.0f, t_pair = 0.0f;
      const ConvImg im = conv_img(ws.feat[0], nullptr, nullptr, nullptr, nullptr, nullptr, ws.t0, hp, wp);
      NV_TRY(time_launch(s, 3, &t_fused, [&] { return launch_resblock(ctx->blocks[0], ctx->blocks[1], ft, im, s); }));
      const ConvImg ia = conv_img(ws.feat[0], nullptr, nullptr, nullptr, nullptr, nullptr, ws.t0, hp, wp);
      const ConvImg ib = conv_img(ws.t0, nullptr, nullptr, nullptr, nullptr, ws.feat[0], ws.u, hp, wp);
      NV_TRY(time_launch(s, 3, &t_pair, [&] {
        const hipError_t e = launch_conv(ctx->blocks[0], CONV_BULK, EPI_LRELU, ft, ctx->tune.pb_block, ia, C, 0, s);
        if (e != hipSuccess) return e;
        return launch_conv(ctx->blocks[1], CONV_BULK, EPI_RES, ft, ctx->tune.pb_block, ib, C, 0, s);
      }));
      ctx->tune.fused = t_fused < t_pair;
      snprintf(buf, sizeof buf, "resblock: fused=%.1fus pair=%.1fus -> %s; ", 1000.0f * t_fused, 1000.0f * t_pair,
               ctx->tune.fused ? "fused" : "pair");
      rep += buf;
    }
    NV_TRY(order_end(ctx->ws_ord, s));
    if (cache) {
      if (FILE* f = fopen(cache, "a")) {
        fprintf(f, "%s | %d %d %d %d %d %d\n", key, ctx->tune.pb_block, ctx->tune.pb_up, ctx->tune.pb_dcn,
                ctx->tune.off1, ctx->tune.off2, ctx->tune.fused);
        fclose(f);
      }
    }
  } else {
    rep = "from cache: ";
    rep += key;
  }
  char tail[160];
  snprintf(tail, sizeof tail, " [block %s%s, up %s, dcn %s, off1 %s, off2 %s; LDS limit %d]",
           tile_name(ctx->tune.pb_block).c_str(), resblocks_fused(ctx) ? " (fused blocks)" : "",
           tile_name(ctx->tune.pb_up).c_str(), dcn_tile_name(ctx->tune.pb_dcn).c_str(), tile_name(ctx->tune.off1).c_str(),
           tile_name(ctx->tune.off2).c_str(), lds_limit());
  rep += tail;
  if (ctx->batch && ctx->batch->exec) {   // the recorded graph holds the old tile shapes
    HIP_TRY(hipDeviceSynchronize());
    (void)hipGraphExecDestroy(ctx->batch->exec);
    ctx->batch->exec = nullptr;
  }
  if (report && report_len > 0) snprintf(report, report_len, "%s", rep.c_str());
  return NV_OK;
}

// ----------------------------------------------------------- kernel timing ----

static const char* const kKindNames[NV_K_COUNT] = {"unpack", "scene", "conv_in", "conv_block", "off1",
                                                   "off2",   "dcn",   "up",      "hr",         "pack",
                                                   "resblock", "pool", "cascade"};

extern "C" const char* nv_profile_kind_name(int32_t kind) {
  return kind >= 0 && kind < NV_K_COUNT ? kKindNames[kind] : "";
}

extern "C" nv_status nv_profile_enable(nv_context* ctx, int32_t on) {
  if (!ctx) return fail(NV_E_INVALID, "NULL argument");
  if (on) {
    HIP_TRY(hipDeviceSynchronize());
    ctx->prof.recs.clear();
    ctx->prof.used = 0;
  }
  ctx->prof.on = on != 0;
  return NV_OK;
}

extern "C" nv_status nv_profile_read(nv_context* ctx, int64_t* launches, double* ms) {
  if (!ctx || !launches || !ms) return fail(NV_E_INVALID, "NULL argument");
  for (int k = 0; k < NV_K_COUNT; ++k) {
    launches[k] = 0;
    ms[k] = 0.0;
  }
  for (const auto& r : ctx->prof.recs) {
    HIP_TRY(hipEventSynchronize(r.b));
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    launches[r.kind] += 1;
    ms[r.kind] += (double)t;
  }
  return NV_OK;
}

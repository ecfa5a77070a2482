// Host runtime and C-ABI of the enhancement library: argument validation, weight
// repacking, the per-context workspace, the frame-group pipeline and clip streams.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
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

struct LayerSpec {
  const char* name;
  int cout, cin;
};

std::vector<LayerSpec> layer_specs(const nv_net_config& c) {
  const int C = c.channels, G = c.offset_groups;
  std::vector<LayerSpec> v;
  v.push_back({"conv_in", C, 3});
  for (int r = 0; r < c.res_blocks; ++r) {
    v.push_back({"block.a", C, C});
    v.push_back({"block.b", C, C});
  }
  v.push_back({"off1", C, 2 * C});
  v.push_back({"off2", 27 * G, C});
  v.push_back({"dcn", C, 2 * C});
  v.push_back({"up", 4 * C, C});
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
  if (G <= 0 || (2 * c->channels) % G != 0 || ((2 * c->channels) / G) % 4 != 0)
    return fail(NV_E_INVALID, "offset_groups must divide 2C into groups of a multiple of 4 channels");
  if (c->scale != 2) return fail(NV_E_UNSUPPORTED, "only scale 2 is implemented");
  if (c->align != 8) return fail(NV_E_UNSUPPORTED, "only align 8 is implemented");
  if (c->flags != (NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE))
    return fail(NV_E_UNSUPPORTED, "only Interpolation|Extra frame|Double frame (n = 1) is implemented");
  if (c->precision != NV_FP32)
    return fail(c->precision >= 0 && c->precision <= 3 ? NV_E_UNSUPPORTED : NV_E_INVALID,
                "precision %d not available", c->precision);
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
  return NV_OK;
}

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
  return r;
}

int round_up(int v, int a) { return (v + a - 1) / a * a; }

template <class T>
hipError_t dev_alloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T) > 0 ? count * sizeof(T) : 16);
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

// ------------------------------------------------------------------ context ----

struct Workspace {
  int hp = 0, wp = 0;
  float* t0 = nullptr;    // extract temporaries [hp][wp][C]
  float* o1 = nullptr;    // offset-head hidden  [hp][wp][C]
  float* offs = nullptr;  // offsets + mask      [hp][wp][ldo]
  float* fmid = nullptr;  // aligned features    [hp][wp][C]
  float* u = nullptr;     // HR features         [2hp][2wp][C]
  float* hr = nullptr;    // HR RGB              [3][2hp][2wp]
  float* rgb[2] = {nullptr, nullptr};  // group inputs [3][hp][wp]
  float* feat[2] = {nullptr, nullptr}; // group features [hp][wp][C]
  size_t bytes = 0;
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

struct nv_context {
  int device = 0;
  Profiler prof;
  nv_net_config cfg{};
  int C = 0, G = 0, ldo = 0;
  PlainConv conv_in, hr;
  std::vector<PackedConv> blocks;   // a, b per residual block
  PackedConv off1, off2, dcn, up;
  Workspace ws;
  std::vector<void*> allocs;
};

namespace {

// A-operand fragments of one conv for the MFMA kernels: element
//   frag[(((tap * NKG + kg) * obtot + ob) * 64 + lane) * 4 + kk]
//     = W[o = rowmap(16*ob + lane%16)][c = 16*kg + 4*(lane/16) + kk][tap]
// and bias[r] = b[rowmap(r)], zero for padded rows.  rowmap is the identity except for
// the pixel-shuffle conv, whose A row 16*ob + t carries channel 16*(ob/4) + t of
// sub-pixel ob%4, i.e. original output channel 4*(16*(ob/4) + t) + ob%4.
nv_status pack_conv(nv_context* ctx, const float* w, const float* b, int cout, int cin,
                    bool shuffle, PackedConv* out) {
  const int obtot = (cout + 15) / 16;
  const int nkg = cin / 16;
  std::vector<float> frag((size_t)9 * nkg * obtot * 64 * 4, 0.0f);
  std::vector<float> bias((size_t)obtot * 16, 0.0f);
  auto rowmap = [&](int r) -> int {
    if (!shuffle) return r;
    const int ob = r / 16, t = r % 16;
    return 4 * (16 * (ob / 4) + t) + (ob % 4);
  };
  for (int tap = 0; tap < 9; ++tap)
    for (int kg = 0; kg < nkg; ++kg)
      for (int ob = 0; ob < obtot; ++ob)
        for (int lane = 0; lane < 64; ++lane)
          for (int kk = 0; kk < 4; ++kk) {
            const int r = 16 * ob + lane % 16;
            if (r >= cout) continue;
            const int o = rowmap(r);
            const int c = 16 * kg + 4 * (lane / 16) + kk;
            frag[((((size_t)tap * nkg + kg) * obtot + ob) * 64 + lane) * 4 + kk] =
                w[((size_t)o * cin + c) * 9 + tap];
          }
  for (int r = 0; r < cout; ++r) bias[r] = b[rowmap(r)];
  out->cin = cin;
  out->cout = cout;
  out->obtot = obtot;
  HIP_TRY(dev_alloc(&out->frag, frag.size()));
  ctx->allocs.push_back(out->frag);
  HIP_TRY(dev_alloc(&out->bias, bias.size()));
  ctx->allocs.push_back(out->bias);
  HIP_TRY(hipMemcpy(out->frag, frag.data(), frag.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(out->bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

nv_status upload(nv_context* ctx, const std::vector<float>& v, float** out) {
  HIP_TRY(dev_alloc(out, v.size()));
  ctx->allocs.push_back(*out);
  HIP_TRY(hipMemcpy(*out, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  return NV_OK;
}

void free_workspace(Workspace& ws) {
  dev_free(ws.t0);
  dev_free(ws.o1);
  dev_free(ws.offs);
  dev_free(ws.fmid);
  dev_free(ws.u);
  dev_free(ws.hr);
  for (int i = 0; i < 2; ++i) {
    dev_free(ws.rgb[i]);
    dev_free(ws.feat[i]);
  }
  ws.hp = ws.wp = 0;
  ws.bytes = 0;
}

// Grows the workspace to (hp, wp).  Freeing memory that queued work may still read
// requires the device to be idle first.
nv_status ensure_workspace(nv_context* ctx, int hp, int wp) {
  Workspace& ws = ctx->ws;
  if (ws.hp >= hp && ws.wp >= wp && ws.t0) return NV_OK;
  const int nh = hp > ws.hp ? hp : ws.hp, nw = wp > ws.wp ? wp : ws.wp;
  if (ws.t0) {
    HIP_TRY(hipDeviceSynchronize());
    free_workspace(ws);
  }
  const size_t px = (size_t)nh * nw, C = ctx->C;
  Workspace n;
  n.hp = nh;
  n.wp = nw;
  HIP_TRY(dev_alloc(&n.t0, px * C));
  ws = n;  // from here on free_workspace() releases whatever was allocated
  HIP_TRY(dev_alloc(&ws.o1, px * C));
  HIP_TRY(dev_alloc(&ws.offs, px * ctx->ldo));
  HIP_TRY(dev_alloc(&ws.fmid, px * C));
  HIP_TRY(dev_alloc(&ws.u, 4 * px * C));
  HIP_TRY(dev_alloc(&ws.hr, 12 * px));
  for (int i = 0; i < 2; ++i) {
    HIP_TRY(dev_alloc(&ws.rgb[i], 3 * px));
    HIP_TRY(dev_alloc(&ws.feat[i], px * C));
  }
  ws.bytes = 4 * px * (C * 4 + ctx->ldo + 4 * C + 12 + 6 + 2 * C);
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

nv_status extract_impl(nv_context* ctx, const float* rgb, int hp, int wp, float* feat,
                       hipStream_t s) {
  NV_TRY(ensure_workspace(ctx, hp, wp));
  const int C = ctx->C;
  NV_TRY(timed(ctx, NV_K_CONV_IN, s, "conv_in",
               [&] { return launch_conv_in(ctx->conv_in, rgb, feat, hp, wp, s); }));
  for (int r = 0; r < ctx->cfg.res_blocks; ++r) {
    NV_TRY(timed(ctx, NV_K_CONV_BLOCK, s, "block.a", [&] {
      return launch_conv(ctx->blocks[2 * r], EPI_LRELU, feat, nullptr, nullptr, nullptr, nullptr,
                         nullptr, ctx->ws.t0, C, hp, wp, 0, s);
    }));
    NV_TRY(timed(ctx, NV_K_CONV_BLOCK, s, "block.b", [&] {
      return launch_conv(ctx->blocks[2 * r + 1], EPI_RES, ctx->ws.t0, nullptr, nullptr, nullptr,
                         nullptr, feat, feat, C, hp, wp, 0, s);
    }));
  }
  return NV_OK;
}

// After HR output t has been written to hr_out[t], pack it into pack_out[t] when given.
nv_status fuse_impl(nv_context* ctx, const float* rgb_a, const float* rgb_b, const float* fa,
                    const float* fb, int hp, int wp, const uint32_t* sel, uint32_t mask,
                    float* const hr_out[3], float* offs_out, float* fmid_out,
                    const nv_format* pack_fmt, const nv_planes* const pack_out[3], hipStream_t s) {
  NV_TRY(ensure_workspace(ctx, hp, wp));
  Workspace& ws = ctx->ws;
  const int C = ctx->C, G = ctx->G;
  float* offs = offs_out ? offs_out : ws.offs;
  float* fmid = fmid_out ? fmid_out : ws.fmid;
  if (mask & 2u) {
    NV_TRY(timed(ctx, NV_K_OFF1, s, "off1", [&] {
      return launch_conv(ctx->off1, EPI_LRELU, fa, fb, sel, nullptr, fa, nullptr, ws.o1, C, hp, wp, 0, s);
    }));
    NV_TRY(timed(ctx, NV_K_OFF2, s, "off2", [&] {
      return launch_conv(ctx->off2, EPI_OFFSET, ws.o1, nullptr, nullptr, nullptr, nullptr, nullptr, offs,
                         ctx->ldo, hp, wp, 18 * G, s);
    }));
    NV_TRY(timed(ctx, NV_K_DCN, s, "dcn",
                 [&] { return launch_dcn(ctx->dcn, fa, fb, sel, offs, ctx->ldo, G, fmid, hp, wp, s); }));
  }
  for (int t = 0; t < 3; ++t) {
    if (!(mask & (1u << t))) continue;
    const float* g = t == 0 ? fa : (t == 1 ? fmid : fb);
    const float* alt = t == 2 ? fa : nullptr;
    const int tsel = t == 0 ? 0 : (t == 1 ? 2 : 1);
    NV_TRY(timed(ctx, NV_K_UP, s, "up", [&] {
      return launch_conv(ctx->up, EPI_SHUFFLE, g, nullptr, sel, alt, nullptr, nullptr, ws.u, 4 * C, hp,
                         wp, 0, s);
    }));
    float* hr = hr_out && hr_out[t] ? hr_out[t] : ws.hr;
    NV_TRY(timed(ctx, NV_K_HR, s, "hr",
                 [&] { return launch_hr(ctx->hr, ws.u, rgb_a, rgb_b, sel, tsel, hr, hp, wp, s); }));
    if (pack_fmt && pack_out && pack_out[t]) {
      const FrameOut fo = to_frame_out(pack_fmt, pack_out[t]);
      NV_TRY(timed(ctx, NV_K_PACK, s, "pack", [&] { return launch_pack(fo, hr, 2 * hp, 2 * wp, s); }));
    }
  }
  return NV_OK;
}

nv_format out_format(const nv_format* f) {
  nv_format o = *f;
  o.width *= 2;
  o.height *= 2;
  return o;
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
  nv_context* ctx = new (std::nothrow) nv_context;
  if (!ctx) return fail(NV_E_NOMEM, "host allocation failed");
  ctx->device = device;
  ctx->cfg = *cfg;
  ctx->C = cfg->channels;
  ctx->G = cfg->offset_groups;
  ctx->ldo = 16 * ((27 * ctx->G + 15) / 16);
  const auto specs = layer_specs(*cfg);
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
      // fragments of the response matrix: row r = 3*tap + o (27 rows, padded to 32)
      //   frag[((cg*2 + ob)*64 + lane)*4 + kk] = w[o][c = 16cg + 4(lane/16) + kk][tap]
      const int nkg = L.cin / 16;
      std::vector<float> w4((size_t)nkg * 2 * 64 * 4, 0.0f);
      for (int cg = 0; cg < nkg; ++cg)
        for (int ob = 0; ob < 2; ++ob)
          for (int lane = 0; lane < 64; ++lane)
            for (int kk = 0; kk < 4; ++kk) {
              const int r = 16 * ob + lane % 16;
              if (r >= 27) continue;
              const int tap = r / 3, o = r % 3, c = 16 * cg + 4 * (lane / 16) + kk;
              w4[(((size_t)cg * 2 + ob) * 64 + lane) * 4 + kk] = w[((size_t)o * L.cin + c) * 9 + tap];
            }
      ctx->hr.cin = L.cin;
      ctx->hr.cout = 3;
      st = upload(ctx, w4, &ctx->hr.w);
      if (st == NV_OK) st = upload(ctx, std::vector<float>(b, b + 3), &ctx->hr.b);
    } else {
      PackedConv pc;
      st = pack_conv(ctx, w, b, L.cout, L.cin, nm == "up", &pc);
      if (nm == "block.a" || nm == "block.b") ctx->blocks.push_back(pc);
      else if (nm == "off1") ctx->off1 = pc;
      else if (nm == "off2") ctx->off2 = pc;
      else if (nm == "dcn") ctx->dcn = pc;
      else if (nm == "up") ctx->up = pc;
    }
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
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
  delete ctx;
  return NV_OK;
}

extern "C" int32_t nv_feature_elem_bytes(const nv_context* ctx) {
  if (!ctx) return 0;
  return ctx->cfg.precision == NV_FP32 ? 4 : 2;
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
  if (rh < fmt->height || rw < fmt->width || rh > 2 * kMaxDim || rw > 2 * kMaxDim)
    return fail(NV_E_INVALID, "RGB size %dx%d smaller than the frame", rw, rh);
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
  const Frame c = to_frame(fmt, cur);
  Frame p = to_frame(fmt, prev);
  return check_launch(launch_scene(c, prev ? &p : nullptr, d_hist_prev, to_rule(params), external_cut,
                                   d_sad, d_hist, d_hd, d_cut, (hipStream_t)stream),
                      "scene");
}

// --------------------------------------------------------------- network ----

static nv_status check_dims(int hp, int wp) {
  if (hp <= 0 || wp <= 0 || hp % 8 || wp % 8 || hp > kMaxDim || wp > kMaxDim)
    return fail(NV_E_INVALID, "padded size %dx%d must be positive multiples of 8", wp, hp);
  return NV_OK;
}

extern "C" nv_status nv_extract(nv_context* ctx, const float* d_rgb, int32_t hp, int32_t wp,
                                void* d_feat, void* stream) {
  if (!ctx || !d_rgb || !d_feat) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_dims(hp, wp));
  return extract_impl(ctx, d_rgb, hp, wp, static_cast<float*>(d_feat), (hipStream_t)stream);
}

extern "C" nv_status nv_fuse(nv_context* ctx, const float* d_rgb_a, const float* d_rgb_b,
                             const void* d_feat_a, const void* d_feat_b, int32_t hp, int32_t wp,
                             const uint32_t* d_sel, uint32_t out_mask, float* const d_hr[3],
                             float* d_offsets, void* d_fmid, void* stream) {
  if (!ctx || !d_rgb_a || !d_rgb_b || !d_feat_a || !d_feat_b) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_dims(hp, wp));
  if (out_mask == 0 || out_mask > 7) return fail(NV_E_INVALID, "out_mask must be in 1..7");
  for (int t = 0; t < 3; ++t)
    if ((out_mask & (1u << t)) && (!d_hr || !d_hr[t])) return fail(NV_E_INVALID, "d_hr[%d] is NULL", t);
  return fuse_impl(ctx, d_rgb_a, d_rgb_b, static_cast<const float*>(d_feat_a),
                   static_cast<const float*>(d_feat_b), hp, wp, d_sel, out_mask, d_hr, d_offsets,
                   static_cast<float*>(d_fmid), nullptr, nullptr, (hipStream_t)stream);
}

extern "C" nv_status nv_enhance_group(nv_context* ctx, const nv_format* fmt, const nv_planes in[2],
                                      const nv_planes out[3], void* stream) {
  if (!ctx || !in || !out) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_format(fmt, "input"));
  NV_TRY(check_planes(fmt, &in[0], "input 0"));
  NV_TRY(check_planes(fmt, &in[1], "input 1"));
  const nv_format of = out_format(fmt);
  NV_TRY(check_format(&of, "output"));
  for (int i = 0; i < 3; ++i) NV_TRY(check_planes(&of, &out[i], "output"));
  const int hp = round_up(fmt->height, 8), wp = round_up(fmt->width, 8);
  NV_TRY(ensure_workspace(ctx, hp, wp));
  hipStream_t s = (hipStream_t)stream;
  Workspace& ws = ctx->ws;
  for (int i = 0; i < 2; ++i) {
    const Frame f = to_frame(fmt, &in[i]);
    NV_TRY(timed(ctx, NV_K_UNPACK, s, "unpack", [&] { return launch_unpack(f, ws.rgb[i], hp, wp, s); }));
    NV_TRY(extract_impl(ctx, ws.rgb[i], hp, wp, ws.feat[i], s));
  }
  const nv_planes* po[3] = {&out[0], &out[1], &out[2]};
  return fuse_impl(ctx, ws.rgb[0], ws.rgb[1], ws.feat[0], ws.feat[1], hp, wp, nullptr, 7u, nullptr,
                   nullptr, nullptr, &of, po, s);
}

// ---------------------------------------------------------------- streams ----

struct nv_stream {
  nv_context* ctx = nullptr;
  nv_format fmt{};
  nv_format ofmt{};
  SceneRule rule{};
  int hp = 0, wp = 0;
  int64_t t = 0;                 // frames pushed
  float* rgb[2] = {nullptr, nullptr};
  float* feat[2] = {nullptr, nullptr};
  void* luma[2] = {nullptr, nullptr};   // copy of each frame's luma plane (scene metric)
  int64_t luma_pitch = 0;
  uint32_t* hist = nullptr;      // [2][64]
  uint64_t* sad = nullptr;
  uint32_t* hd = nullptr;
  uint32_t* cuts = nullptr;      // [kCutRing]
  size_t bytes = 0;
};

static size_t stream_bytes(const nv_context* ctx, const nv_format* f) {
  const size_t hp = round_up(f->height, 8), wp = round_up(f->width, 8);
  const size_t bps = f->bits == 8 ? 1 : 2;
  return 2 * (3 * hp * wp * 4 + hp * wp * (size_t)ctx->C * 4 + (size_t)f->width * f->height * bps) +
         2 * 64 * 4 + 8 + 4 + (size_t)kCutRing * 4;
}

static void stream_free(nv_stream* s) {
  for (int i = 0; i < 2; ++i) {
    dev_free(s->rgb[i]);
    dev_free(s->feat[i]);
    if (s->luma[i]) (void)hipFree(s->luma[i]);
    s->luma[i] = nullptr;
  }
  dev_free(s->hist);
  dev_free(s->sad);
  dev_free(s->hd);
  dev_free(s->cuts);
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
  NV_TRY(check_scene_params(params));
  nv_stream* s = new (std::nothrow) nv_stream;
  if (!s) return fail(NV_E_NOMEM, "host allocation failed");
  s->ctx = ctx;
  s->fmt = *fmt;
  s->ofmt = out_format(fmt);
  s->rule = to_rule(params);
  s->hp = round_up(fmt->height, 8);
  s->wp = round_up(fmt->width, 8);
  const size_t px = (size_t)s->hp * s->wp;
  s->luma_pitch = (int64_t)fmt->width * (fmt->bits == 8 ? 1 : 2);
  hipError_t e = hipSuccess;
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = dev_alloc(&s->rgb[i], 3 * px);
    if (e == hipSuccess) e = dev_alloc(&s->feat[i], px * ctx->C);
    if (e == hipSuccess) e = hipMalloc(&s->luma[i], (size_t)s->luma_pitch * fmt->height);
  }
  if (e == hipSuccess) e = dev_alloc(&s->hist, 128);
  if (e == hipSuccess) e = dev_alloc(&s->sad, 1);
  if (e == hipSuccess) e = dev_alloc(&s->hd, 1);
  if (e == hipSuccess) e = dev_alloc(&s->cuts, kCutRing);
  if (e != hipSuccess) {
    stream_free(s);
    delete s;
    return fail(e == hipErrorOutOfMemory ? NV_E_NOMEM : NV_E_DEVICE, "stream allocation: %s",
                hipGetErrorString(e));
  }
  s->bytes = stream_bytes(ctx, fmt);
  nv_status st = ensure_workspace(ctx, s->hp, s->wp);
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
  return fuse_impl(s->ctx, s->rgb[slot_a], s->rgb[slot_b], s->feat[slot_a], s->feat[slot_b], s->hp,
                   s->wp, cut_b, 3u, nullptr, nullptr, nullptr, &s->ofmt, po, hs);
}

extern "C" nv_status nv_stream_push(nv_stream* s, const nv_planes* frame, int32_t external_cut,
                                    const nv_planes out[2], int32_t* n_out, void* stream) {
  if (!s || !n_out) return fail(NV_E_INVALID, "NULL argument");
  NV_TRY(check_planes(&s->fmt, frame, "frame"));
  if (external_cut < -1 || external_cut > 1) return fail(NV_E_INVALID, "external_cut must be -1, 0 or 1");
  if (s->t > 0) {
    if (!out) return fail(NV_E_INVALID, "out is NULL");
    for (int i = 0; i < 2; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  }
  hipStream_t hs = (hipStream_t)stream;
  const int cur = (int)(s->t & 1), prv = cur ^ 1;
  const Frame f = to_frame(&s->fmt, frame);
  NV_TRY(timed(s->ctx, NV_K_UNPACK, hs, "unpack", [&] { return launch_unpack(f, s->rgb[cur], s->hp, s->wp, hs); }));
  Frame pf = f;
  pf.p[0] = s->luma[prv];
  pf.pitch[0] = s->luma_pitch;
  uint32_t* cut_t = s->cuts + (s->t % kCutRing);
  NV_TRY(timed(s->ctx, NV_K_SCENE, hs, "scene", [&] {
    return launch_scene(f, s->t > 0 ? &pf : nullptr, s->t > 0 ? s->hist + 64 * prv : nullptr, s->rule,
                        external_cut, s->sad, s->hist + 64 * cur, s->hd, cut_t, hs);
  }));
  HIP_TRY(hipMemcpy2DAsync(s->luma[cur], (size_t)s->luma_pitch, frame->data[0],
                           (size_t)frame->pitch_bytes[0], (size_t)s->luma_pitch, (size_t)s->fmt.height,
                           hipMemcpyDeviceToDevice, hs));
  NV_TRY(extract_impl(s->ctx, s->rgb[cur], s->hp, s->wp, s->feat[cur], hs));
  *n_out = 0;
  if (s->t > 0) {
    NV_TRY(emit_group(s, prv, cur, cut_t, out, hs));
    *n_out = 2;
  }
  s->t += 1;
  return NV_OK;
}

extern "C" nv_status nv_stream_end(nv_stream* s, const nv_planes out[2], int32_t* n_out, void* stream) {
  if (!s || !n_out) return fail(NV_E_INVALID, "NULL argument");
  *n_out = 0;
  if (s->t == 0) return NV_OK;
  if (!out) return fail(NV_E_INVALID, "out is NULL");
  for (int i = 0; i < 2; ++i) NV_TRY(check_planes(&s->ofmt, &out[i], "output"));
  const int last = (int)((s->t - 1) & 1);
  NV_TRY(emit_group(s, last, last, nullptr, out, (hipStream_t)stream));
  *n_out = 2;
  return NV_OK;
}

extern "C" nv_status nv_stream_cuts(nv_stream* s, uint32_t* host_cuts, int32_t n, void* stream) {
  if (!s || (!host_cuts && n > 0)) return fail(NV_E_INVALID, "NULL argument");
  if (n < 0 || n > s->t || n > kCutRing) return fail(NV_E_INVALID, "n = %d but %lld frames pushed", n, (long long)s->t);
  if (n == 0) return NV_OK;
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

// ----------------------------------------------------------- kernel timing ----

static const char* const kKindNames[NV_K_COUNT] = {"unpack", "scene", "conv_in", "conv_block", "off1",
                                                   "off2",   "dcn",   "up",      "hr",         "pack"};

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

// Host-only test double of the HIP runtime and of the library's kernel launchers (see
// fake_hip/hip/hip_runtime.h).  Device allocations are host allocations kept in a
// registry; every launcher stub checks that each device pointer it receives lies in a
// live allocation with room for what the real kernel would touch, and counts the
// launch.  Stream, event and graph calls keep just enough state to check the library's
// ordering across streams.
#include "fake_runtime.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

struct ihipStream_t {
  int id;
  bool capturing = false;
};
struct ihipEvent_t {
  hipStream_t stream = nullptr;   // stream of the last record
  long seq = 0;                   // records so far
};
struct ihipGraph {
  int dummy = 0;
};
struct hipGraphExec {
  int dummy = 0;
};

namespace fake {

struct Alloc {
  size_t bytes;
  bool pinned;
};
static std::map<uintptr_t, Alloc>& allocs() {
  static std::map<uintptr_t, Alloc> m;
  return m;
}
static long g_launches = 0, g_bad = 0;
static std::vector<Wait> g_waits;
static std::vector<std::string> g_errors;
static int g_next_stream = 1;

long launches() { return g_launches; }
long bad_pointers() { return g_bad; }
const std::vector<Wait>& waits() { return g_waits; }
void clear_waits() { g_waits.clear(); }
size_t live_bytes() {
  size_t n = 0;
  for (auto& kv : allocs())
    if (!kv.second.pinned) n += kv.second.bytes;
  return n;
}
size_t live_allocations() {
  size_t n = 0;
  for (auto& kv : allocs())
    if (!kv.second.pinned) ++n;
  return n;
}
hipStream_t new_stream() {
  hipStream_t s = nullptr;
  hipStreamCreateWithFlags(&s, 0);
  return s;
}
int stream_id(hipStream_t s) { return s ? s->id : 0; }
const std::vector<std::string>& errors() { return g_errors; }

// p .. p + bytes inside one live allocation
bool in_alloc(const void* p, size_t bytes) {
  if (!p) return false;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto& m = allocs();
  auto it = m.upper_bound(a);
  if (it == m.begin()) return false;
  --it;
  return a >= it->first && a + bytes <= it->first + it->second.bytes;
}

void need(const void* p, size_t bytes, const char* what) {
  if (!in_alloc(p, bytes)) {
    ++g_bad;
    char b[256];
    snprintf(b, sizeof b, "%s: pointer %p with %zu bytes is not inside a live allocation", what, p, bytes);
    g_errors.push_back(b);
  }
}

}  // namespace fake

using fake::need;

// ------------------------------------------------------------------- runtime ----

const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorInvalidValue: return "hipErrorInvalidValue";
    default: return "hipError(fake)";
  }
}

hipError_t hipMalloc(void** p, size_t bytes) {
  void* m = std::calloc(1, bytes ? bytes : 1);
  if (!m) return hipErrorOutOfMemory;
  fake::allocs()[reinterpret_cast<uintptr_t>(m)] = {bytes, false};
  *p = m;
  return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  void* m = std::calloc(1, bytes ? bytes : 1);
  if (!m) return hipErrorOutOfMemory;
  fake::allocs()[reinterpret_cast<uintptr_t>(m)] = {bytes, true};
  *p = m;
  return hipSuccess;
}

static hipError_t release(void* p, bool pinned) {
  if (!p) return hipSuccess;
  auto& m = fake::allocs();
  auto it = m.find(reinterpret_cast<uintptr_t>(p));
  if (it == m.end() || it->second.pinned != pinned) {
    fake::g_errors.push_back("free of a pointer that is not a live allocation");
    ++fake::g_bad;
    return hipErrorInvalidValue;
  }
  m.erase(it);
  std::free(p);
  return hipSuccess;
}

hipError_t hipFree(void* p) { return release(p, false); }
hipError_t hipHostFree(void* p) { return release(p, true); }

hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k) {
  if (k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice) need(dst, bytes, "memcpy dst");
  if (k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice) need(src, bytes, "memcpy src");
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(dst, src, bytes, k);
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                             size_t height, hipMemcpyKind k, hipStream_t) {
  if (height == 0) return hipSuccess;
  if (k == hipMemcpyDeviceToDevice || k == hipMemcpyHostToDevice) need(dst, (height - 1) * dpitch + width, "memcpy2d dst");
  if (k == hipMemcpyDeviceToDevice || k == hipMemcpyDeviceToHost) need(src, (height - 1) * spitch + width, "memcpy2d src");
  for (size_t r = 0; r < height; ++r)
    std::memmove(static_cast<char*>(dst) + r * dpitch, static_cast<const char*>(src) + r * spitch, width);
  return hipSuccess;
}
hipError_t hipMemset(void* p, int v, size_t bytes) {
  need(p, bytes, "memset");
  if (fake::in_alloc(p, bytes)) std::memset(p, v, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t) { return hipMemset(p, v, bytes); }
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t{fake::g_next_stream++};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  fake::g_waits.push_back({fake::stream_id(s), fake::stream_id(e->stream), e->seq});
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  s->capturing = true;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  s->capturing = false;
  *g = new ihipGraph;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new ihipEvent_t;
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->stream = s;
  e->seq += 1;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, void*, void*, size_t) {
  *x = new hipGraphExec;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
// the library's static device arrays are host statics here: their address is the symbol's
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) {
  ++fake::g_launches;
  return hipSuccess;
}

// ------------------------------------------------------------ launcher stubs ----

namespace nv {

static size_t px(int h, int w) { return (size_t)h * (size_t)w; }

Inv make_inv(int, int, int) { return Inv{}; }
Fwd make_fwd(int, int, int) { return Fwd{}; }

static void need_frame(const Frame& f, const char* what) {
  const int bps = f.bits == 8 ? 1 : 2;
  for (int i = 0; i < 3; ++i) {
    const int w = (i == 0 || f.chroma == 444) ? f.w : f.w / 2;
    const int h = (i == 0 || f.chroma == 444) ? f.h : f.h / 2;
    need(f.p[i], (size_t)(h - 1) * f.pitch[i] + (size_t)w * bps, what);
  }
}

hipError_t launch_unpack(const Frame& f, float* rgb, int hp, int wp, hipStream_t) {
  ++fake::g_launches;
  need_frame(f, "unpack input");
  need(rgb, 12 * px(hp, wp), "unpack rgb");
  return hipSuccess;
}

hipError_t launch_pack(const FrameOut& f, const float* rgb, int rh, int rw, hipStream_t) {
  ++fake::g_launches;
  Frame fr;
  for (int i = 0; i < 3; ++i) {
    fr.p[i] = f.p[i];
    fr.pitch[i] = f.pitch[i];
  }
  fr.w = f.w;
  fr.h = f.h;
  fr.bits = f.bits;
  fr.chroma = f.chroma;
  need_frame(fr, "pack output");
  need(rgb, 12 * px(rh, rw), "pack rgb");
  return hipSuccess;
}

hipError_t launch_scene(const SceneJob& j, bool, hipStream_t) {
  ++fake::g_launches;
  need_frame(j.cur, "scene frame");
  need(j.sad, 8, "scene sad");
  need(j.hist, 256, "scene hist");
  need(j.hd, 4, "scene hd");
  need(j.cut, 4, "scene cut");
  if (j.hist_prev) need(j.hist_prev, 256, "scene previous hist");
  if (j.hist_save) need(j.hist_save, 256, "scene hist save");
  if (j.luma_save) need(j.luma_save, (size_t)j.luma_save_pitch * j.cur.h, "scene luma save");
  return hipSuccess;
}

hipError_t launch_unpack_batch(const UnpackJob* jobs, const int* count, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(UnpackJob), "unpack jobs");
  need(count, 8, "unpack count");
  return hipSuccess;
}
hipError_t launch_pack_batch(const PackJob* jobs, const int* count, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(PackJob), "pack jobs");
  need(count, 8, "pack count");
  return hipSuccess;
}
hipError_t launch_scene_batch(const SceneJob* jobs, const int* count, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(SceneJob), "scene jobs");
  need(count, 8, "scene count");
  return hipSuccess;
}

int bulk_tile_lds(int, int, int) { return 1024; }
int lds_limit() { return 163840; }
bool lds_weight_tiles() { return false; }
int conv_ob(int, int, int obtot, int, int) { return obtot % 4 == 0 ? 4 : (obtot % 2 == 0 ? 2 : 1); }
bool resblock_supported(const PackedConv&, const PackedConv&, int) { return false; }
hipError_t launch_resblock(const PackedConv&, const PackedConv&, int, const ConvImg&, hipStream_t) {
  return hipErrorInvalidValue;
}

hipError_t launch_conv_in(const PlainConv& L, int tout, const float* rgb, void* dst, int H, int W, hipStream_t) {
  ++fake::g_launches;
  need(L.w, (size_t)L.cout * 27 * 4, "conv_in weights");
  need(rgb, 12 * px(H, W), "conv_in rgb");
  need(dst, px(H, W) * L.cout * dtype_bytes(tout), "conv_in dst");
  return hipSuccess;
}

hipError_t launch_conv(const PackedConv& P, int role, int epi, int tin, int, const ConvImg& im, int ldy, int,
                       hipStream_t) {
  ++fake::g_launches;
  need(P.frag, 16, "conv weights");
  need(P.bias, (size_t)P.obtot * 64, "conv bias");
  const size_t n = px(im.H, im.W);
  const size_t inb = role == CONV_OFF2 ? 4 : dtype_bytes(tin);
  const int cin = role == CONV_OFF1 ? P.cin / 2 : (P.tc == DT_F16 && role == CONV_OFF2 ? P.cin / 2 : P.cin);
  need(im.src0, n * cin * inb, "conv src0");
  if (role == CONV_OFF1) need(im.src1, n * cin * inb, "conv src1");
  if (im.alt0) need(im.alt0, n * cin * inb, "conv alt0");
  if (im.alt1) need(im.alt1, n * cin * inb, "conv alt1");
  if (im.sel) need(im.sel, 4, "conv sel");
  const size_t outb = role == CONV_BULK ? dtype_bytes(tin) : 4;
  if (epi == EPI_SHUFFLE) need(im.dst, 4 * n * (P.cout / 4) * outb, "conv dst (shuffle)");
  else need(im.dst, n * ldy * outb, "conv dst");
  if (epi == EPI_RES) need(im.res, n * ldy * outb, "conv res");
  return hipSuccess;
}

hipError_t launch_dcn(const PackedConv& P, int tf, int, const DcnImg& im, int ldo, int, hipStream_t) {
  ++fake::g_launches;
  const size_t n = px(im.H, im.W), fb = dtype_bytes(tf);
  need(P.frag, 16, "dcn weights");
  need(im.fa, n * P.cout * fb, "dcn fa");
  need(im.fb, n * P.cout * fb, "dcn fb");
  need(im.offs, n * ldo * 4, "dcn offsets");
  need(im.dst, n * P.cout * fb, "dcn dst");
  if (im.sel) need(im.sel, 4, "dcn sel");
  return hipSuccess;
}

hipError_t launch_hr(const PackedConv& P, int tu, const HrImg& im, hipStream_t) {
  ++fake::g_launches;
  const size_t n = px(im.H, im.W);
  need(P.frag, 16, "hr weights");
  need(im.u, 4 * n * P.cin * dtype_bytes(tu), "hr u");
  need(im.rgb_a, 12 * n, "hr rgb_a");
  need(im.rgb_b, 12 * n, "hr rgb_b");
  need(im.dst, 48 * n, "hr dst");
  if (im.sel) need(im.sel, 4, "hr sel");
  return hipSuccess;
}

hipError_t launch_pool2(int t, const void* src, void* dst, int H2, int W2, int C, hipStream_t) {
  ++fake::g_launches;
  const size_t n = px(H2, W2) * C * dtype_bytes(t);
  need(src, 4 * n, "pool src");
  need(dst, n, "pool dst");
  return hipSuccess;
}

hipError_t launch_up2_add(int t, void* dst, int ldd, const void* src, int lds, int H, int W, int nch, float,
                          hipStream_t) {
  ++fake::g_launches;
  if (nch > ldd || nch > lds) return hipErrorInvalidValue;
  need(dst, px(H, W) * ldd * dtype_bytes(t), "cascade dst");
  need(src, px(H / 2, W / 2) * lds * dtype_bytes(t), "cascade src");
  return hipSuccess;
}

hipError_t launch_amax(int dt, const void* x, size_t n, uint32_t* amax, hipStream_t) {
  ++fake::g_launches;
  need(x, n * dtype_bytes(dt), "amax input");
  need(amax, 4, "amax out");
  return hipSuccess;
}

hipError_t launch_qscale(const uint32_t* amax, const float* ws, float* os, float* ainv, int rows, hipStream_t) {
  ++fake::g_launches;
  need(amax, 4, "qscale amax");
  need(ws, (size_t)rows * 4, "qscale wscale");
  need(os, (size_t)rows * 4, "qscale oscale");
  need(ainv, 4, "qscale ainv");
  return hipSuccess;
}

hipError_t launch_conv_in_batch(const PlainConv&, int, const ConvInImg* jobs, const int* count, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(ConvInImg), "conv_in jobs");
  need(count, 8, "conv_in count");
  return hipSuccess;
}
hipError_t launch_conv_batch(const PackedConv&, int, int, int, int, const ConvImg* jobs, const int* count, int, int,
                             hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(ConvImg), "conv jobs");
  need(count, 8, "conv count");
  return hipSuccess;
}
hipError_t launch_dcn_batch(const PackedConv&, int, int, const DcnImg* jobs, const int* count, int, int, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(DcnImg), "dcn jobs");
  need(count, 8, "dcn count");
  return hipSuccess;
}
hipError_t launch_hr_batch(const PackedConv&, int, const HrImg* jobs, const int* count, hipStream_t) {
  ++fake::g_launches;
  need(jobs, sizeof(HrImg), "hr jobs");
  need(count, 8, "hr count");
  return hipSuccess;
}

}  // namespace nv

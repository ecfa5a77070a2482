// Host-only checks of the library's host runtime (api.cpp) against the fake HIP runtime,
// built with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_build.py.
// Each case prints "ok <name>" or "FAIL <name>: <why>"; the exit status is the number
// of failures (a sanitizer report aborts the run).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nnvisr.h"
#include "fake_runtime.h"

static int g_fail = 0;
static std::string g_case;

#define EXPECT(cond)                                                                         \
  do {                                                                                       \
    if (!(cond)) {                                                                           \
      std::printf("FAIL %s: %s (line %d; last error: %s)\n", g_case.c_str(), #cond, __LINE__, \
                  nv_last_error());                                                          \
      ++g_fail;                                                                              \
      return;                                                                                \
    }                                                                                        \
  } while (0)

static void run(const char* name, void (*fn)()) {
  g_case = name;
  const int before = g_fail;
  const long bad = fake::bad_pointers();
  fn();
  if (g_fail == before && fake::bad_pointers() != bad) {
    std::printf("FAIL %s: a launch or copy received a pointer outside every live allocation:\n", name);
    for (const auto& e : fake::errors()) std::printf("    %s\n", e.c_str());
    ++g_fail;
  } else if (g_fail == before) {
    std::printf("ok %s\n", name);
  }
  std::fflush(stdout);
}

static void fault(long long min_bytes) {
  if (min_bytes > 0) {
    const std::string v = std::to_string(min_bytes);
    setenv("NNVISR_FAULT_ALLOC_MIN_BYTES", v.c_str(), 1);
  } else {
    unsetenv("NNVISR_FAULT_ALLOC_MIN_BYTES");
  }
}

static nv_net_config cfg32() {
  nv_net_config c{};
  c.channels = 32;
  c.res_blocks = 1;
  c.offset_groups = 8;
  c.scale = 2;
  c.align = 8;
  c.flags = NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE;
  c.precision = NV_FP32;
  return c;
}

static std::vector<float> weights(const nv_net_config& c) {
  std::vector<float> w(nv_weight_count(&c));
  unsigned x = 12345u;
  for (auto& v : w) {
    x = x * 1664525u + 1013904223u;
    v = ((x >> 9) & 0xFFFF) / 65536.0f * 0.02f - 0.01f;
  }
  return w;
}

static nv_context* make_ctx() {
  const nv_net_config c = cfg32();
  const std::vector<float> w = weights(c);
  nv_context* ctx = nullptr;
  if (nv_context_create(0, &c, w.data(), w.size(), &ctx) != NV_OK) return nullptr;
  return ctx;
}

struct Frame {
  nv_planes p{};
  void alloc(int w, int h, int chroma = 420) {
    const int cw = chroma == 420 ? w / 2 : w, ch = chroma == 420 ? h / 2 : h;
    hipMalloc(&p.data[0], (size_t)w * h);
    hipMalloc(&p.data[1], (size_t)cw * ch);
    hipMalloc(&p.data[2], (size_t)cw * ch);
    p.pitch_bytes[0] = w;
    p.pitch_bytes[1] = p.pitch_bytes[2] = cw;
  }
  void free_() {
    for (auto& d : p.data) hipFree(d);
  }
};

static nv_format fmt(int w, int h) {
  nv_format f{};
  f.width = w;
  f.height = h;
  f.bits = 8;
  f.chroma = 420;
  return f;
}

// ---------------------------------------------------------------- cases ----

static void validation() {
  nv_context* out = reinterpret_cast<nv_context*>(0x1);
  nv_net_config c = cfg32();
  std::vector<float> w = weights(c);
  EXPECT(nv_context_create(0, nullptr, w.data(), w.size(), &out) == NV_E_INVALID && out == nullptr);
  EXPECT(nv_context_create(0, &c, w.data(), w.size() - 1, &out) == NV_E_INVALID);
  EXPECT(nv_context_create(1, &c, w.data(), w.size(), &out) == NV_E_INVALID);
  c.channels = 48;
  EXPECT(nv_context_create(0, &c, w.data(), w.size(), &out) == NV_E_INVALID);
  c = cfg32();
  c.scale = 3;
  EXPECT(nv_context_create(0, &c, w.data(), w.size(), &out) == NV_E_UNSUPPORTED);
  nv_context* ctx = make_ctx();
  EXPECT(ctx != nullptr);
  nv_format f = fmt(63, 64);
  nv_stream* s = nullptr;
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_E_INVALID && s == nullptr);
  f = fmt(64, 64);
  f.bits = 9;
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_E_INVALID);
  f = fmt(64, 64);
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_OK);
  Frame fr;
  fr.alloc(64, 64);
  nv_planes bad = fr.p;
  bad.pitch_bytes[0] = 63;
  int32_t n = -7;
  const long launches = fake::launches();
  EXPECT(nv_stream_push(s, &bad, -1, nullptr, &n, nullptr) == NV_E_INVALID);
  EXPECT(nv_stream_push(s, &fr.p, 2, nullptr, &n, nullptr) == NV_E_INVALID);
  EXPECT(fake::launches() == launches);            // nothing enqueued
  uint32_t cut = 0;
  EXPECT(nv_stream_cuts(s, &cut, 1, nullptr) == NV_E_INVALID);   // still no frame pushed
  EXPECT(nv_stream_push(s, &fr.p, -1, nullptr, &n, nullptr) == NV_OK && n == 0);
  EXPECT(nv_stream_cuts(s, &cut, 1, nullptr) == NV_OK);
  nv_stream_close(s);
  fr.free_();
  nv_context_destroy(ctx);
}

// Workspace growth that fails part way (the offsets buffer, the third of its
// allocations) must leave no half-built workspace behind: the failing call returns
// NV_E_NOMEM and frees what it allocated, and the next call allocates afresh.
static void workspace_nomem_then_retry() {
  nv_context* ctx = make_ctx();
  EXPECT(ctx != nullptr);
  const int hp = 64, wp = 64, C = 32, ldo = 224;
  const size_t offs_bytes = (size_t)hp * wp * ldo * 4;
  std::vector<void*> bufs;
  auto dev = [&](size_t bytes) {
    void* p = nullptr;
    hipMalloc(&p, bytes);
    bufs.push_back(p);
    return p;
  };
  float* rgb_a = (float*)dev(12 * hp * wp);
  float* rgb_b = (float*)dev(12 * hp * wp);
  void* fa = dev((size_t)hp * wp * C * 4);
  void* fb = dev((size_t)hp * wp * C * 4);
  float* hr[3] = {(float*)dev(48 * hp * wp), (float*)dev(48 * hp * wp), (float*)dev(48 * hp * wp)};
  const size_t live = fake::live_allocations();
  fault((long long)offs_bytes);
  EXPECT(nv_fuse(ctx, rgb_a, rgb_b, fa, fb, hp, wp, nullptr, 7u, hr, nullptr, nullptr, nullptr) == NV_E_NOMEM);
  EXPECT(fake::live_allocations() == live);        // the partial workspace was released
  EXPECT(nv_fuse(ctx, rgb_a, rgb_b, fa, fb, hp, wp, nullptr, 7u, hr, nullptr, nullptr, nullptr) == NV_E_NOMEM);
  fault(0);
  EXPECT(nv_fuse(ctx, rgb_a, rgb_b, fa, fb, hp, wp, nullptr, 7u, hr, nullptr, nullptr, nullptr) == NV_OK);
  EXPECT(nv_extract(ctx, rgb_a, hp, wp, fa, nullptr) == NV_OK);
  nv_context_destroy(ctx);
  for (void* p : bufs) hipFree(p);
}

// A stream whose open fails for lack of memory leaves nothing allocated; once memory is
// available the same context opens it and runs a clip.
static void stream_open_nomem_then_clip() {
  nv_context* ctx = make_ctx();
  EXPECT(ctx != nullptr);
  const nv_format f = fmt(64, 64);
  const size_t live = fake::live_allocations();
  fault((long long)64 * 64 * 224 * 4);
  nv_stream* s = nullptr;
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_E_NOMEM && s == nullptr);
  EXPECT(fake::live_allocations() == live);
  fault(0);
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_OK);
  Frame in[3], out[2];
  for (auto& x : in) x.alloc(64, 64);
  for (auto& x : out) x.alloc(128, 128);
  nv_planes po[2] = {out[0].p, out[1].p};
  for (int t = 0; t < 3; ++t) {
    int32_t n = -1;
    EXPECT(nv_stream_push(s, &in[t].p, -1, po, &n, nullptr) == NV_OK && n == (t ? 2 : 0));
  }
  int32_t n = -1;
  EXPECT(nv_stream_end(s, po, &n, nullptr) == NV_OK && n == 2);
  nv_stream_close(s);
  for (auto& x : in) x.free_();
  for (auto& x : out) x.free_();
  nv_context_destroy(ctx);
}

// A batch whose ring growth fails returns NV_E_NOMEM without advancing the stream; the
// stream still takes pushes, and the same batch succeeds once memory is available.
static void batch_nomem_stream_usable() {
  nv_context* ctx = make_ctx();
  EXPECT(ctx != nullptr);
  const nv_format f = fmt(64, 64);
  nv_stream* s = nullptr;
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s) == NV_OK);
  Frame in[4], out[8];
  for (auto& x : in) x.alloc(64, 64);
  for (auto& x : out) x.alloc(128, 128);
  nv_planes fr[3] = {in[0].p, in[1].p, in[2].p};
  nv_planes po[8];
  for (int i = 0; i < 8; ++i) po[i] = out[i].p;
  int32_t n_out = -1;
  nv_batch_req r{};
  r.stream = s;
  r.n_frames = 3;
  r.frames = fr;
  r.out = po;
  r.n_out = &n_out;
  fault(1);                                        // every device allocation fails
  EXPECT(nv_enhance_batch(ctx, &r, 1, nullptr) == NV_E_NOMEM);
  uint32_t cut = 0;
  EXPECT(nv_stream_cuts(s, &cut, 1, nullptr) == NV_E_INVALID);   // no frame counted
  fault(0);
  int32_t n = -1;
  EXPECT(nv_stream_push(s, &in[3].p, -1, po, &n, nullptr) == NV_OK && n == 0);
  // the batch state itself fails to build: the context stays without one and retries
  r.n_frames = 1;
  r.frames = &fr[0];
  fault(1);
  EXPECT(nv_enhance_batch(ctx, &r, 1, nullptr) == NV_E_NOMEM);
  fault(0);
  size_t bb = 1;
  EXPECT(nv_batch_footprint(ctx, &bb) == NV_OK && bb == 0);
  r.n_frames = 3;
  r.frames = fr;
  r.end_of_clip = 1;
  EXPECT(nv_enhance_batch(ctx, &r, 1, nullptr) == NV_OK && n_out == 8);
  EXPECT(nv_batch_footprint(ctx, &bb) == NV_OK && bb > 0);
  nv_stream_close(s);
  for (auto& x : in) x.free_();
  for (auto& x : out) x.free_();
  nv_context_destroy(ctx);
}

// The waits between the caller's HIP streams a and b (the context's own fork / join with
// its side stream is internal to one call and ordered by the caller's stream).
static std::vector<fake::Wait> caller_waits(int a, int b) {
  std::vector<fake::Wait> v;
  for (const auto& w : fake::waits())
    if ((w.waiter == a || w.waiter == b) && (w.recorded_on == a || w.recorded_on == b)) v.push_back(w);
  return v;
}

// Calls on different HIP streams: the second stream waits for the event recorded after
// the last call that used the shared workspace or the clip stream's state.
static void ordering_across_streams() {
  nv_context* ctx = make_ctx();
  EXPECT(ctx != nullptr);
  const nv_format f = fmt(64, 64);
  nv_stream *s1 = nullptr, *s2 = nullptr;
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s1) == NV_OK);
  EXPECT(nv_stream_open(ctx, &f, nullptr, &s2) == NV_OK);
  hipStream_t A = fake::new_stream(), B = fake::new_stream();
  const int a = fake::stream_id(A), b = fake::stream_id(B);
  Frame in[4], out[2];
  for (auto& x : in) x.alloc(64, 64);
  for (auto& x : out) x.alloc(128, 128);
  nv_planes po[2] = {out[0].p, out[1].p};
  int32_t n = 0;
  fake::clear_waits();
  EXPECT(nv_stream_push(s1, &in[0].p, -1, po, &n, A) == NV_OK);
  EXPECT(caller_waits(a, b).empty());                   // first use: nothing to wait for
  EXPECT(nv_stream_push(s2, &in[1].p, -1, po, &n, B) == NV_OK);
  // s2's own state is new; the context workspace was last used on A
  EXPECT(caller_waits(a, b).size() == 1 && caller_waits(a, b)[0].waiter == b && caller_waits(a, b)[0].recorded_on == a);
  fake::clear_waits();
  EXPECT(nv_stream_push(s2, &in[2].p, -1, po, &n, B) == NV_OK);
  EXPECT(caller_waits(a, b).empty());                   // same stream: ordered by the stream
  EXPECT(nv_stream_push(s1, &in[3].p, -1, po, &n, B) == NV_OK);
  // s1 was last pushed on A: B waits for it (the workspace was last used on B itself)
  EXPECT(caller_waits(a, b).size() == 1 && caller_waits(a, b)[0].waiter == b && caller_waits(a, b)[0].recorded_on == a);
  fake::clear_waits();
  uint32_t cuts[2];
  EXPECT(nv_stream_cuts(s1, cuts, 2, A) == NV_OK);
  EXPECT(caller_waits(a, b).size() == 1 && caller_waits(a, b)[0].waiter == a && caller_waits(a, b)[0].recorded_on == b);
  nv_stream_close(s1);
  nv_stream_close(s2);
  hipStreamDestroy(A);
  hipStreamDestroy(B);
  for (auto& x : in) x.free_();
  for (auto& x : out) x.free_();
  nv_context_destroy(ctx);
}

static void nothing_leaks() {
  EXPECT(fake::live_allocations() == 0);
}

int main() {
  run("validation_before_any_work", validation);
  run("workspace_nomem_then_retry", workspace_nomem_then_retry);
  run("stream_open_nomem_then_clip", stream_open_nomem_then_clip);
  run("batch_nomem_stream_usable", batch_nomem_stream_usable);
  run("ordering_across_streams", ordering_across_streams);
  run("nothing_leaks", nothing_leaks);
  std::printf("failures %d\n", g_fail);
  return g_fail;
}

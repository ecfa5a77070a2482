// Scenario driver of the CPU simulation build (tests/test_cpusim.py): runs the library's
// C-ABI on host buffers that stand in for device memory and writes the results as raw
// files for the test to compare with the FP64 oracle.
//
//   driver net DIR C R G PREC H W   reads DIR/weights.f32, DIR/rgb_a.f32, DIR/rgb_b.f32
//                                   (planar float [3][H][W]); writes fa, fb (features),
//                                   offs (float [H][W][ldo]), fmid, hr0, hr1, hr2
//                                   (float [3][2H][2W]) as DIR/<name>.bin
#include <hip/hip_runtime.h>
#include <nnvisr.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

static std::vector<char> read_file(const std::string& p) {
  std::vector<char> v;
  FILE* f = fopen(p.c_str(), "rb");
  if (!f) {
    fprintf(stderr, "cannot read %s\n", p.c_str());
    exit(2);
  }
  fseek(f, 0, SEEK_END);
  v.resize(ftell(f));
  fseek(f, 0, SEEK_SET);
  if (!v.empty() && fread(v.data(), 1, v.size(), f) != v.size()) exit(2);
  fclose(f);
  return v;
}

static void write_file(const std::string& p, const void* d, size_t n) {
  FILE* f = fopen(p.c_str(), "wb");
  if (!f || fwrite(d, 1, n, f) != n) {
    fprintf(stderr, "cannot write %s\n", p.c_str());
    exit(2);
  }
  fclose(f);
}

#define CHECK(x)                                                                   \
  do {                                                                             \
    nv_status s_ = (x);                                                            \
    if (s_ != NV_OK) {                                                             \
      fprintf(stderr, "%s failed: %d %s\n", #x, (int)s_, nv_last_error());        \
      exit(1);                                                                     \
    }                                                                              \
  } while (0)

static void* dev(size_t bytes, const void* init = nullptr) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) exit(2);
  if (init) memcpy(p, init, bytes);
  return p;
}

static int run_net(int argc, char** argv) {
  if (argc < 9) return 2;
  const std::string dir = argv[2];
  nv_net_config cfg{};
  cfg.channels = atoi(argv[3]);
  cfg.res_blocks = atoi(argv[4]);
  cfg.offset_groups = atoi(argv[5]);
  cfg.scale = 2;
  cfg.align = 8;
  cfg.flags = NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE;
  cfg.precision = atoi(argv[6]);
  const int H = atoi(argv[7]), W = atoi(argv[8]);
  const std::vector<char> wb = read_file(dir + "/weights.f32");
  nv_context* ctx = nullptr;
  CHECK(nv_context_create(0, &cfg, reinterpret_cast<const float*>(wb.data()), wb.size() / 4, &ctx));
  if (getenv("NNVISR_TUNE_CACHE")) {   // tiles forced through the tuner's cache file
    char rep[512];
    CHECK(nv_autotune(ctx, H, W, nullptr, rep, sizeof rep));
    fprintf(stderr, "%s\n", rep);
  }
  const std::vector<char> ra = read_file(dir + "/rgb_a.f32"), rb = read_file(dir + "/rgb_b.f32");
  const size_t px = (size_t)H * W, fe = (size_t)nv_feature_elem_bytes(ctx), C = cfg.channels;
  const int ldo = 16 * ((27 * cfg.offset_groups + 15) / 16);
  float* da = static_cast<float*>(dev(12 * px, ra.data()));
  float* db = static_cast<float*>(dev(12 * px, rb.data()));
  void* fa = dev(px * C * fe);
  void* fb = dev(px * C * fe);
  float* offs = static_cast<float*>(dev(px * ldo * 4));
  void* fmid = dev(px * C * fe);
  float* hr[3];
  for (int t = 0; t < 3; ++t) hr[t] = static_cast<float*>(dev(48 * px));
  fprintf(stderr, "net C=%d R=%d G=%d prec=%d %dx%d: extract\n", cfg.channels, cfg.res_blocks, cfg.offset_groups,
          cfg.precision, W, H);
  CHECK(nv_extract(ctx, da, H, W, fa, nullptr));
  CHECK(nv_extract(ctx, db, H, W, fb, nullptr));
  fprintf(stderr, "fuse\n");
  CHECK(nv_fuse(ctx, da, db, fa, fb, H, W, nullptr, 7u, hr, offs, fmid, nullptr));
  write_file(dir + "/fa.bin", fa, px * C * fe);
  write_file(dir + "/fb.bin", fb, px * C * fe);
  write_file(dir + "/offs.bin", offs, px * ldo * 4);
  write_file(dir + "/fmid.bin", fmid, px * C * fe);
  for (int t = 0; t < 3; ++t) write_file(dir + "/hr" + std::to_string(t) + ".bin", hr[t], 48 * px);
  CHECK(nv_context_destroy(ctx));
  for (void* p : {(void*)da, (void*)db, fa, fb, (void*)offs, fmid, (void*)hr[0], (void*)hr[1], (void*)hr[2]})
    hipFree(p);
  fprintf(stderr, "done\n");
  return 0;
}

// One 8-bit 4:2:0 frame of pseudo-random codes (planes padded to a 64-byte pitch).
struct HostFrame {
  std::vector<uint8_t> p[3];
  int64_t pitch[3];
};
static HostFrame make_frame(int w, int h, uint32_t seed) {
  HostFrame f;
  uint32_t x = seed * 2654435761u + 12345u;
  for (int i = 0; i < 3; ++i) {
    const int pw = i ? w / 2 : w, ph = i ? h / 2 : h;
    f.pitch[i] = (pw + 63) / 64 * 64;
    f.p[i].assign((size_t)f.pitch[i] * ph, 0);
    for (int y = 0; y < ph; ++y)
      for (int c = 0; c < pw; ++c) {
        x = x * 1664525u + 1013904223u;
        f.p[i][(size_t)y * f.pitch[i] + c] = (uint8_t)(16 + (x >> 24) % 220);
      }
  }
  return f;
}
static nv_planes to_dev(const HostFrame& f) {
  nv_planes p;
  for (int i = 0; i < 3; ++i) {
    p.data[i] = dev(f.p[i].size(), f.p[i].data());
    p.pitch_bytes[i] = f.pitch[i];
  }
  return p;
}
static nv_planes out_planes(int w, int h) {
  HostFrame z;
  for (int i = 0; i < 3; ++i) {
    const int pw = i ? w / 2 : w, ph = i ? h / 2 : h;
    z.pitch[i] = (pw + 63) / 64 * 64;
    z.p[i].assign((size_t)z.pitch[i] * ph, 0);
  }
  return to_dev(z);
}

// driver static C R G PREC: nv_enhance_group_static against nv_enhance_group on two
// groups in a row (the second smaller), bit for bit, and a group too large for the
// static scratch rejected with NV_E_INVALID.
static int run_static(int argc, char** argv) {
  if (argc < 6) return 2;
  nv_net_config cfg{};
  cfg.channels = atoi(argv[2]);
  cfg.res_blocks = atoi(argv[3]);
  cfg.offset_groups = atoi(argv[4]);
  cfg.scale = 2;
  cfg.align = 8;
  cfg.flags = NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE;
  cfg.precision = atoi(argv[5]);
  std::vector<float> w(nv_weight_count(&cfg));
  uint32_t x = 7;
  for (float& v : w) {
    x = x * 1664525u + 1013904223u;
    v = ((int)(x >> 9) - (1 << 22)) / (float)(1 << 22) * 0.05f;
  }
  nv_context* ctx = nullptr;
  CHECK(nv_context_create(0, &cfg, w.data(), w.size(), &ctx));
  const int sizes[2][2] = {{40, 24}, {24, 16}};
  for (int k = 0; k < 2; ++k) {
    const int W = sizes[k][0], H = sizes[k][1];
    nv_format fmt{W, H, 8, 420};
    const nv_planes in[2] = {to_dev(make_frame(W, H, 1 + k)), to_dev(make_frame(W, H, 11 + k))};
    nv_planes ref[3], got[3];
    for (int t = 0; t < 3; ++t) {
      ref[t] = out_planes(2 * W, 2 * H);
      got[t] = out_planes(2 * W, 2 * H);
    }
    CHECK(nv_enhance_group(ctx, &fmt, in, ref, nullptr));
    CHECK(nv_enhance_group_static(ctx, &fmt, in, got, nullptr));
    for (int t = 0; t < 3; ++t)
      for (int i = 0; i < 3; ++i) {
        const size_t n = (size_t)ref[t].pitch_bytes[i] * (i ? H : 2 * H);
        if (memcmp(ref[t].data[i], got[t].data[i], n) != 0) {
          fprintf(stderr, "static: group %dx%d output %d plane %d differs\n", W, H, t, i);
          return 1;
        }
      }
    fprintf(stderr, "static: group %dx%d bit-identical\n", W, H);
  }
  nv_format big{4096, 4096, 8, 420};
  const nv_planes bin[2] = {out_planes(4096, 4096), out_planes(4096, 4096)};
  nv_planes bo[3];
  for (int t = 0; t < 3; ++t) bo[t] = out_planes(8192, 8192);
  const nv_status st = nv_enhance_group_static(ctx, &big, bin, bo, nullptr);
  if (st != NV_E_INVALID) {
    fprintf(stderr, "static: 4096x4096 group returned %d, expected NV_E_INVALID\n", (int)st);
    return 1;
  }
  fprintf(stderr, "static: oversized group rejected: %s\n", nv_last_error());
  CHECK(nv_context_destroy(ctx));
  fprintf(stderr, "static ok\n");
  return 0;
}

// driver unpack|pack DIR W H BITS CHROMA MATRIX RANGE SITING: the pixel-format stages of
// one frame.  Planes are DIR/{y,u,v}.bin, tightly packed (1 or 2 bytes per sample); R'G'B'
// is DIR/rgb.f32, planar float [3][hp][wp] (unpack: hp, wp the sizes rounded up to 8;
// pack: hp = H, wp = W rounded up to 4).
static int run_pixel(int argc, char** argv, bool unpack) {
  if (argc < 10) return 2;
  const std::string dir = argv[2];
  nv_format fmt{atoi(argv[3]), atoi(argv[4]), atoi(argv[5]), atoi(argv[6]), atoi(argv[7]), atoi(argv[8]),
                atoi(argv[9])};
  const int W = fmt.width, H = fmt.height, bps = fmt.bits == 8 ? 1 : 2;
  const int cw = fmt.chroma == 420 ? W / 2 : W, ch = fmt.chroma == 420 ? H / 2 : H;
  nv_planes pl;
  const char* names[3] = {"y", "u", "v"};
  for (int i = 0; i < 3; ++i) {
    const int pw = i ? cw : W, ph = i ? ch : H;
    pl.pitch_bytes[i] = (int64_t)pw * bps;
    if (unpack) {
      const std::vector<char> d = read_file(dir + "/" + names[i] + ".bin");
      pl.data[i] = dev(d.size(), d.data());
    } else {
      pl.data[i] = dev((size_t)pw * ph * bps);
    }
  }
  if (unpack) {
    const int hp = (H + 7) / 8 * 8, wp = (W + 7) / 8 * 8;
    float* rgb = static_cast<float*>(dev((size_t)12 * hp * wp));
    CHECK(nv_unpack(&fmt, &pl, rgb, hp, wp, nullptr));
    write_file(dir + "/rgb.f32", rgb, (size_t)12 * hp * wp);
    hipFree(rgb);
  } else {
    const int rw = (W + 3) / 4 * 4;
    const std::vector<char> d = read_file(dir + "/rgb.f32");
    if (d.size() != (size_t)12 * H * rw) return 2;
    float* rgb = static_cast<float*>(dev(d.size(), d.data()));
    CHECK(nv_pack(&fmt, rgb, H, rw, &pl, nullptr));
    for (int i = 0; i < 3; ++i) {
      const int pw = i ? cw : W, ph = i ? ch : H;
      write_file(dir + "/" + names[i] + ".bin", pl.data[i], (size_t)pw * ph * bps);
    }
    hipFree(rgb);
  }
  for (int i = 0; i < 3; ++i) hipFree(pl.data[i]);
  return 0;
}

// driver clip C R G N B W H FRAMES S1 S2 ...: a clip of FRAMES pseudo-random 8-bit 4:2:0
// frames whose scenes start at the listed frames (external cut flags, metric off) through
// nv_clip_* with n = N, b = B and through nv_stream_*; the outputs must be bit-identical.
// Prints "trace:" and the clip's trace values, then "clip ok".
static int run_clip(int argc, char** argv) {
  if (argc < 9) return 2;
  nv_net_config cfg{};
  cfg.channels = atoi(argv[2]);
  cfg.res_blocks = atoi(argv[3]);
  cfg.offset_groups = atoi(argv[4]);
  cfg.scale = 2;
  cfg.align = 8;
  cfg.flags = NV_FLAG_INTERP | NV_FLAG_EXTRA | NV_FLAG_DOUBLE;
  const int n = atoi(argv[5]), b = atoi(argv[6]), W = atoi(argv[7]), H = atoi(argv[8]), T = atoi(argv[9]);
  std::vector<int> starts;
  for (int i = 10; i < argc; ++i) starts.push_back(atoi(argv[i]));
  std::vector<float> w(nv_weight_count(&cfg));
  uint32_t x = 11;
  for (float& v : w) {
    x = x * 1664525u + 1013904223u;
    v = ((int)(x >> 9) - (1 << 22)) / (float)(1 << 22) * 0.05f;
  }
  nv_context* ctx = nullptr;
  CHECK(nv_context_create(0, &cfg, w.data(), w.size(), &ctx));
  nv_format fmt{W, H, 8, 420};
  nv_scene_params sp{24, 1, 4, 0};
  std::vector<nv_planes> frames;
  for (int t = 0; t < T; ++t) frames.push_back(to_dev(make_frame(W, H, 100 + t)));
  auto ext = [&](int t) {
    for (int s0 : starts)
      if (s0 == t) return 1;
    return 0;
  };
  nv_clip* clip = nullptr;
  CHECK(nv_clip_open(ctx, &fmt, &sp, n, b, &clip));
  const int cap = 2 * n * b;
  std::vector<nv_planes> got;
  std::vector<nv_planes> room(cap);
  auto fresh = [&]() {
    for (int i = 0; i < cap; ++i) room[i] = out_planes(2 * W, 2 * H);
  };
  for (int t = 0; t < T; ++t) {
    fresh();
    int32_t k = 0;
    CHECK(nv_clip_push(clip, &frames[t], ext(t), room.data(), cap, &k, nullptr));
    for (int i = 0; i < k; ++i) got.push_back(room[i]);
  }
  fresh();
  int32_t k = 0;
  CHECK(nv_clip_end(clip, room.data(), cap, &k, nullptr));
  for (int i = 0; i < k; ++i) got.push_back(room[i]);
  // the same frames through a clip stream (n = 1, no frame store)
  nv_stream* st = nullptr;
  CHECK(nv_stream_open(ctx, &fmt, &sp, &st));
  std::vector<nv_planes> ref;
  for (int t = 0; t <= T; ++t) {
    nv_planes o[2] = {out_planes(2 * W, 2 * H), out_planes(2 * W, 2 * H)};
    int32_t m = 0;
    if (t < T) CHECK(nv_stream_push(st, &frames[t], ext(t), o, &m, nullptr));
    else CHECK(nv_stream_end(st, o, &m, nullptr));
    for (int i = 0; i < m; ++i) ref.push_back(o[i]);
  }
  if (got.size() != ref.size() || (int)got.size() != 2 * T) {
    fprintf(stderr, "clip: %zu outputs, stream %zu, expected %d\n", got.size(), ref.size(), 2 * T);
    return 1;
  }
  for (size_t i = 0; i < got.size(); ++i)
    for (int pl = 0; pl < 3; ++pl) {
      const size_t bytes = (size_t)got[i].pitch_bytes[pl] * (pl ? H : 2 * H);
      if (memcmp(got[i].data[pl], ref[i].data[pl], bytes) != 0) {
        fprintf(stderr, "clip: output %zu plane %d differs from the stream's\n", i, pl);
        return 1;
      }
    }
  int32_t len = 0;
  CHECK(nv_clip_trace(clip, nullptr, 0, &len));
  std::vector<int32_t> tr(len);
  CHECK(nv_clip_trace(clip, tr.data(), len, &len));
  printf("trace:");
  for (int32_t v : tr) printf(" %d", v);
  printf("\n");
  CHECK(nv_clip_close(clip));
  CHECK(nv_stream_close(st));
  CHECK(nv_context_destroy(ctx));
  printf("clip ok\n");
  return 0;
}

// driver task DIR C R G SCALE SCALE_V FLAGS W H T: a clip stream of T 8-bit 4:2:0 frames
// (DIR/f<t>_{y,u,v}.bin, tight planes) with weights DIR/weights.f32 for a network of the
// given scale factors and flags; writes the emitted frames as DIR/o<k>_{y,u,v}.bin and
// prints "outputs <count>".
static int run_task(int argc, char** argv) {
  if (argc < 12) return 2;
  const std::string dir = argv[2];
  nv_net_config cfg{};
  cfg.channels = atoi(argv[3]);
  cfg.res_blocks = atoi(argv[4]);
  cfg.offset_groups = atoi(argv[5]);
  cfg.scale = atoi(argv[6]);
  cfg.scale_v = atoi(argv[7]);
  cfg.align = 8;
  cfg.flags = (uint32_t)atoi(argv[8]);
  const int W = atoi(argv[9]), H = atoi(argv[10]), T = atoi(argv[11]);
  cfg.levels = argc > 12 ? atoi(argv[12]) : 0;
  const std::vector<char> wb = read_file(dir + "/weights.f32");
  nv_context* ctx = nullptr;
  CHECK(nv_context_create(0, &cfg, reinterpret_cast<const float*>(wb.data()), wb.size() / 4, &ctx));
  nv_format fmt{W, H, 8, 420};
  nv_scene_params sp{24, 1, 4, 1};
  nv_stream* st = nullptr;
  CHECK(nv_stream_open(ctx, &fmt, &sp, &st));
  const int sv = cfg.scale_v ? cfg.scale_v : cfg.scale, sh = cfg.scale;
  const int OW = W * sh, OH = H * sv;
  const char* names[3] = {"y", "u", "v"};
  int k = 0;
  auto save = [&](const nv_planes& o) {
    for (int i = 0; i < 3; ++i) {
      const int pw = i ? OW / 2 : OW, ph = i ? OH / 2 : OH;
      std::vector<uint8_t> buf((size_t)pw * ph);
      for (int y = 0; y < ph; ++y)
        memcpy(&buf[(size_t)y * pw], static_cast<char*>(o.data[i]) + (size_t)y * o.pitch_bytes[i], pw);
      write_file(dir + "/o" + std::to_string(k) + "_" + names[i] + ".bin", buf.data(), buf.size());
    }
    ++k;
  };
  for (int t = 0; t <= T; ++t) {
    nv_planes o[2] = {out_planes(OW, OH), out_planes(OW, OH)};
    int32_t m = 0;
    if (t < T) {
      nv_planes in;
      for (int i = 0; i < 3; ++i) {
        const std::vector<char> d = read_file(dir + "/f" + std::to_string(t) + "_" + names[i] + ".bin");
        in.data[i] = dev(d.size(), d.data());
        in.pitch_bytes[i] = i ? W / 2 : W;
      }
      CHECK(nv_stream_push(st, &in, -1, o, &m, nullptr));
    } else {
      CHECK(nv_stream_end(st, o, &m, nullptr));
    }
    for (int i = 0; i < m; ++i) save(o[i]);
  }
  printf("outputs %d\n", k);
  CHECK(nv_stream_close(st));
  CHECK(nv_context_destroy(ctx));
  return 0;
}

int main(int argc, char** argv) {
  if (argc >= 2 && strcmp(argv[1], "task") == 0) return run_task(argc, argv);
  if (argc >= 2 && strcmp(argv[1], "clip") == 0) return run_clip(argc, argv);
  if (argc >= 2 && strcmp(argv[1], "unpack") == 0) return run_pixel(argc, argv, true);
  if (argc >= 2 && strcmp(argv[1], "pack") == 0) return run_pixel(argc, argv, false);
  if (argc >= 2 && strcmp(argv[1], "net") == 0) return run_net(argc, argv);
  if (argc >= 2 && strcmp(argv[1], "static") == 0) return run_static(argc, argv);
  fprintf(stderr, "usage: driver net DIR C R G PREC H W | static C R G PREC | unpack|pack DIR W H BITS CHROMA MATRIX RANGE SITING\n");
  return 2;
}

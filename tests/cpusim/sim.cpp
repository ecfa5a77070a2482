// CPU simulation of the HIP runtime and device for the library's kernels (test build
// only, see hip/hip_runtime.h).  Work-items run as fibers with a hand-written x86-64
// context switch; the scheduler resumes every ready fiber in work-item order until it
// blocks (barrier, wave operation) or ends, then releases the barrier or computes the
// wave operation once every live participant has arrived.  When nothing can proceed,
// the states of all work-items are printed and the process exits with status 3.
#include <hip/hip_runtime.h>
#include <sys/mman.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size) __attribute__((weak));
void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old)
    __attribute__((weak));
void __asan_unpoison_memory_region(void const volatile* addr, size_t size) __attribute__((weak));
void nvsim_switch(void** save_sp, void* load_sp);
}

// Saves the callee-saved registers, MXCSR and the x87 control word on the current stack,
// stores the stack pointer in *save_sp, and resumes the context whose stack pointer is
// load_sp.
__asm__(
    ".text\n"
    ".globl nvsim_switch\n"
    ".type nvsim_switch,@function\n"
    "nvsim_switch:\n"
    "  pushq %rbp\n"
    "  pushq %rbx\n"
    "  pushq %r12\n"
    "  pushq %r13\n"
    "  pushq %r14\n"
    "  pushq %r15\n"
    "  subq $8, %rsp\n"
    "  stmxcsr (%rsp)\n"
    "  fnstcw 4(%rsp)\n"
    "  movq %rsp, (%rdi)\n"
    "  movq %rsi, %rsp\n"
    "  ldmxcsr (%rsp)\n"
    "  fldcw 4(%rsp)\n"
    "  addq $8, %rsp\n"
    "  popq %r15\n"
    "  popq %r14\n"
    "  popq %r13\n"
    "  popq %r12\n"
    "  popq %rbx\n"
    "  popq %rbp\n"
    "  ret\n"
    ".size nvsim_switch, .-nvsim_switch\n");

struct ihipStream_t {
  bool capturing = false;
  std::vector<std::function<void()>>* rec = nullptr;
};
struct ihipEvent_t {
  int dummy = 0;
};
struct ihipGraph {
  std::vector<std::function<void()>> ops;
};
struct hipGraphExec {
  std::vector<std::function<void()>> ops;
};

namespace nvsim {

nvsim_uint3 g_thread, g_block;
dim3 g_block_dim, g_grid_dim;

namespace {

constexpr size_t kStack = 512 * 1024;
constexpr size_t kGuard = 4096;

enum State { READY, AT_BARRIER, AT_WAVE, DONE };
enum Op {
  OP_NONE,
  OP_MFMA4,
  OP_MFMA16_F16,
  OP_MFMA16_BF16,
  OP_MFMA32_F16,
  OP_MFMA32_BF16,
  OP_MFMA_F8,
  OP_SHFL,
  OP_RFL
};
const char* op_name(int op) {
  static const char* n[] = {"none", "mfma_16x16x4_f32", "mfma_16x16x32_f16", "mfma_16x16x32_bf16",
                            "mfma_32x32x16_f16", "mfma_32x32x16_bf16", "mfma_scale_16x16x128_f8", "shfl_xor",
                            "readfirstlane"};
  return n[op];
}

// per-lane operands and result of a wave operation
struct LaneIO {
  int op = OP_NONE;
  uint8_t a[32], b[32];
  float acc[16];
  float res[16];
  uint64_t v = 0, vres = 0;
  int mask = 0, width = 64;
  int fa = 0, fb = 0, sa = 127, sb = 127;
};

struct Fiber {
  void* sp = nullptr;
  char* mem = nullptr;    // mapping: guard page + stack
  State st = READY;
  void* fake = nullptr;
};

struct BlockRun {
  std::vector<Fiber> f;
  std::vector<LaneIO> io;
  int n = 0, cur = -1;
  void* sched_sp = nullptr;
  const void* main_bottom = nullptr;
  size_t main_size = 0;
  const std::function<void()>* body = nullptr;
};

BlockRun R;
std::vector<char*> g_stacks;

char* stack_mem(int i) {
  while ((int)g_stacks.size() <= i) {
    void* m = mmap(nullptr, kStack + kGuard, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1,
                   0);
    if (m == MAP_FAILED) {
      fprintf(stderr, "nvsim: cannot map a fiber stack\n");
      exit(2);
    }
    mprotect(m, kGuard, PROT_NONE);
    g_stacks.push_back(static_cast<char*>(m));
  }
  return g_stacks[i];
}

void set_thread(int t) {
  g_thread.x = t % g_block_dim.x;
  g_thread.y = (t / g_block_dim.x) % g_block_dim.y;
  g_thread.z = t / (g_block_dim.x * g_block_dim.y);
}

// switch from the running fiber back to the scheduler
void to_scheduler(bool dying) {
  Fiber& me = R.f[R.cur];
  if (__sanitizer_start_switch_fiber) __sanitizer_start_switch_fiber(dying ? nullptr : &me.fake, R.main_bottom, R.main_size);
  nvsim_switch(&me.sp, R.sched_sp);
  if (__sanitizer_finish_switch_fiber) __sanitizer_finish_switch_fiber(me.fake, nullptr, nullptr);
}

void fiber_entry() {
  if (__sanitizer_finish_switch_fiber) __sanitizer_finish_switch_fiber(nullptr, &R.main_bottom, &R.main_size);
  (*R.body)();
  R.f[R.cur].st = DONE;
  to_scheduler(true);
  fprintf(stderr, "nvsim: a finished work-item was resumed\n");
  abort();
}

void run_fiber(int i) {
  R.cur = i;
  set_thread(i);
  Fiber& f = R.f[i];
  if (__sanitizer_start_switch_fiber) __sanitizer_start_switch_fiber(nullptr, f.mem + kGuard, kStack);
  nvsim_switch(&R.sched_sp, f.sp);
  if (__sanitizer_finish_switch_fiber) __sanitizer_finish_switch_fiber(nullptr, nullptr, nullptr);
  R.cur = -1;
}

void start_fiber(int i) {
  Fiber& f = R.f[i];
  f.mem = stack_mem(i);
  char* base = f.mem + kGuard;
  if (__asan_unpoison_memory_region) __asan_unpoison_memory_region(base, kStack);
  char* top = base + kStack;   // 16-byte aligned
  uint64_t* sp = reinterpret_cast<uint64_t*>(top - 72);
  sp[0] = 0x1F80ull | (0x037Full << 32);   // MXCSR, x87 control word
  for (int r = 1; r <= 6; ++r) sp[r] = 0;    // r15 r14 r13 r12 rbx rbp
  sp[7] = reinterpret_cast<uint64_t>(&fiber_entry);
  sp[8] = 0;
  f.sp = sp;
  f.st = READY;
  f.fake = nullptr;
}

[[noreturn]] void hang(const char* why) {
  fprintf(stderr, "nvsim: HANG in workgroup (%u,%u,%u) of grid (%u,%u,%u), block (%u,%u,%u): %s\n", g_block.x,
          g_block.y, g_block.z, g_grid_dim.x, g_grid_dim.y, g_grid_dim.z, g_block_dim.x, g_block_dim.y,
          g_block_dim.z, why);
  for (int w = 0; w * 64 < R.n; ++w) {
    fprintf(stderr, "  wave %d:", w);
    for (int l = 0; l < 64 && w * 64 + l < R.n; ++l) {
      const int i = w * 64 + l;
      const char* s = R.f[i].st == DONE ? "D" : (R.f[i].st == AT_BARRIER ? "B" : (R.f[i].st == AT_WAVE ? "W" : "R"));
      fprintf(stderr, "%s", s);
    }
    fprintf(stderr, "\n");
    for (int l = 0; l < 64 && w * 64 + l < R.n; ++l)
      if (R.f[w * 64 + l].st == AT_WAVE) {
        fprintf(stderr, "    lane %d waits in %s\n", l, op_name(R.io[w * 64 + l].op));
        break;
      }
  }
  fflush(stderr);
  _exit(3);
}

inline float f16_to_f(uint16_t h) {
  _Float16 v;
  memcpy(&v, &h, 2);
  return (float)v;
}
inline float bf16_to_f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
// OCP e4m3 (bias 7, no infinities, 0x7f / 0xff NaN)
inline float e4m3_to_f(uint8_t b) {
  const int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
  float v;
  if (e == 15 && m == 7) v = NAN;
  else if (e == 0) v = ldexpf((float)m, -9);
  else v = ldexpf(1.0f + m / 8.0f, e - 7);
  return s ? -v : v;
}
uint8_t f_to_e4m3(float x) {
  if (std::isnan(x)) return 0x7f;
  const int s = x < 0 ? 0x80 : 0;
  double a = fabs((double)x);
  if (a >= 448.0) return (uint8_t)(s | 0x7e);
  // round to nearest even on the grid of the binade (subnormal step 2^-9)
  int e = a > 0 ? (int)floor(log2(a)) : -10;
  if (e < -6) e = -6;
  const double step = ldexp(1.0, e - 3);
  double q = a / step;
  double r = floor(q);
  const double d = q - r;
  if (d > 0.5 || (d == 0.5 && fmod(r, 2.0) == 1.0)) r += 1.0;
  double v = r * step;
  if (v >= 448.0) return (uint8_t)(s | 0x7e);
  if (v == 0) return (uint8_t)s;
  int ee = (int)floor(log2(v));
  if (ee < -6) {   // subnormal
    return (uint8_t)(s | (int)(v / ldexp(1.0, -9)));
  }
  const int m = (int)((v / ldexp(1.0, ee) - 1.0) * 8.0 + 0.5);
  return (uint8_t)(s | ((ee + 7) << 3) | m);
}

// computes the wave operation of wave w for all of its live lanes
void wave_compute(int w, int op) {
  const int l0 = w * 64;
  const int nl = std::min(64, R.n - l0);
  auto io = [&](int l) -> LaneIO& { return R.io[l0 + l]; };
  auto live = [&](int l) { return l < nl && R.f[l0 + l].st != DONE; };
  switch (op) {
    case OP_MFMA4:
    case OP_MFMA16_F16:
    case OP_MFMA16_BF16:
    case OP_MFMA_F8: {
      // A[i][k]: lane i + 16 (k / KQ) element k % KQ; B[k][j]: lane j + 16 (k / KQ)
      const int KQ = op == OP_MFMA4 ? 1 : (op == OP_MFMA_F8 ? 32 : 8);
      auto elem = [&](const uint8_t* p, int e) -> double {
        if (op == OP_MFMA4) {
          float f;
          memcpy(&f, p, 4);
          return f;
        }
        if (op == OP_MFMA_F8) return e4m3_to_f(p[e]);
        uint16_t h;
        memcpy(&h, p + 2 * e, 2);
        return op == OP_MFMA16_F16 ? f16_to_f(h) : bf16_to_f(h);
      };
      for (int l = 0; l < nl; ++l) {
        if (!live(l)) continue;
        const int j = l & 15, ib = l >> 4;
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * ib + r;
          double s = 0.0;
          for (int q = 0; q < 4; ++q) {
            const int la = i + 16 * q, lb = j + 16 * q;
            if (!live(la) || !live(lb)) continue;
            for (int e = 0; e < KQ; ++e) s += elem(io(la).a, e) * elem(io(lb).b, e);
          }
          if (op == OP_MFMA_F8) s *= ldexp(1.0, io(l).sa - 127) * ldexp(1.0, io(l).sb - 127);
          io(l).res[r] = (float)((double)io(l).acc[r] + s);
        }
      }
      break;
    }
    case OP_MFMA32_F16:
    case OP_MFMA32_BF16: {
      // A[i][k]: lane i + 32 (k / 8) element k % 8; B[k][j]: lane j + 32 (k / 8);
      // D[i][j]: lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4
      auto elem = [&](const uint8_t* p, int e) -> double {
        uint16_t h;
        memcpy(&h, p + 2 * e, 2);
        return op == OP_MFMA32_F16 ? f16_to_f(h) : bf16_to_f(h);
      };
      for (int l = 0; l < nl; ++l) {
        if (!live(l)) continue;
        const int j = l & 31, h = l >> 5;
        for (int v = 0; v < 16; ++v) {
          const int i = 8 * (v / 4) + 4 * h + v % 4;
          double s = 0.0;
          for (int q = 0; q < 2; ++q) {
            const int la = i + 32 * q, lb = j + 32 * q;
            if (!live(la) || !live(lb)) continue;
            for (int e = 0; e < 8; ++e) s += elem(io(la).a, e) * elem(io(lb).b, e);
          }
          io(l).res[v] = (float)((double)io(l).acc[v] + s);
        }
      }
      break;
    }
    case OP_SHFL:
      for (int l = 0; l < nl; ++l) {
        if (!live(l)) continue;
        const int width = io(l).width, src = (l & ~(width - 1)) | ((l ^ io(l).mask) & (width - 1));
        if (!live(src)) hang("lane shuffle reads a lane that has ended");
        io(l).vres = io(src).v;
      }
      break;
    case OP_RFL: {
      int first = -1;
      for (int l = 0; l < nl && first < 0; ++l)
        if (live(l)) first = l;
      for (int l = 0; l < nl; ++l)
        if (live(l)) io(l).vres = io(first).v;
      break;
    }
  }
}

void run_block(const std::function<void()>& body, int n) {
  R.f.assign(n, Fiber{});
  R.io.assign(n, LaneIO{});
  R.n = n;
  R.body = &body;
  for (int i = 0; i < n; ++i) start_fiber(i);
  for (;;) {
    bool progress = false;
    for (int i = 0; i < n; ++i)
      if (R.f[i].st == READY) {
        run_fiber(i);
        progress = true;
      }
    // wave operations whose live lanes have all arrived
    for (int w = 0; w * 64 < n; ++w) {
      const int l0 = w * 64, nl = std::min(64, n - l0);
      int op = OP_NONE, waiting = 0, alive = 0;
      bool mixed = false;
      for (int l = 0; l < nl; ++l) {
        const Fiber& f = R.f[l0 + l];
        if (f.st == DONE) continue;
        ++alive;
        if (f.st == AT_WAVE) {
          ++waiting;
          if (op == OP_NONE) op = R.io[l0 + l].op;
          else if (op != R.io[l0 + l].op) mixed = true;
        }
      }
      if (waiting > 0 && waiting == alive) {
        if (mixed) hang("lanes of one wave wait in different wave operations");
        wave_compute(w, op);
        for (int l = 0; l < nl; ++l)
          if (R.f[l0 + l].st == AT_WAVE) R.f[l0 + l].st = READY;
        progress = true;
      }
    }
    int alive = 0, at_bar = 0;
    for (int i = 0; i < n; ++i) {
      if (R.f[i].st != DONE) ++alive;
      if (R.f[i].st == AT_BARRIER) ++at_bar;
    }
    if (alive == 0) break;
    if (at_bar == alive) {
      for (int i = 0; i < n; ++i)
        if (R.f[i].st == AT_BARRIER) R.f[i].st = READY;
      progress = true;
    }
    if (!progress) hang("no work-item can proceed (barrier not reached by every live work-item, or a wave "
                        "operation not joined by every live lane)");
  }
}

LaneIO& my_io() { return R.io[R.cur]; }

void wave_wait(int op) {
  LaneIO& io = my_io();
  io.op = op;
  R.f[R.cur].st = AT_WAVE;
  to_scheduler(false);
}

}  // namespace

void syncthreads() {
  if (R.cur < 0) {
    fprintf(stderr, "nvsim: __syncthreads outside a kernel\n");
    abort();
  }
  R.f[R.cur].st = AT_BARRIER;
  to_scheduler(false);
}

f32x4_ mfma_f32_16x16x4f32(float a, float b, f32x4_ c, int, int, int) {
  LaneIO& io = my_io();
  memcpy(io.a, &a, 4);
  memcpy(io.b, &b, 4);
  for (int r = 0; r < 4; ++r) io.acc[r] = c[r];
  wave_wait(OP_MFMA4);
  return f32x4_{io.res[0], io.res[1], io.res[2], io.res[3]};
}

template <class V>
static f32x4_ mfma16(V a, V b, f32x4_ c, int op) {
  LaneIO& io = my_io();
  memcpy(io.a, &a, 16);
  memcpy(io.b, &b, 16);
  for (int r = 0; r < 4; ++r) io.acc[r] = c[r];
  wave_wait(op);
  return f32x4_{io.res[0], io.res[1], io.res[2], io.res[3]};
}
f32x4_ mfma_f32_16x16x32_f16(f16x8_ a, f16x8_ b, f32x4_ c, int, int, int) { return mfma16(a, b, c, OP_MFMA16_F16); }
f32x4_ mfma_f32_16x16x32_bf16(bf16x8_ a, bf16x8_ b, f32x4_ c, int, int, int) {
  return mfma16(a, b, c, OP_MFMA16_BF16);
}

template <class V>
static f32x16_ mfma32(V a, V b, f32x16_ c, int op) {
  LaneIO& io = my_io();
  memcpy(io.a, &a, 16);
  memcpy(io.b, &b, 16);
  for (int r = 0; r < 16; ++r) io.acc[r] = c[r];
  wave_wait(op);
  f32x16_ o;
  for (int r = 0; r < 16; ++r) o[r] = io.res[r];
  return o;
}
f32x16_ mfma_f32_32x32x16_f16(f16x8_ a, f16x8_ b, f32x16_ c, int, int, int) { return mfma32(a, b, c, OP_MFMA32_F16); }
f32x16_ mfma_f32_32x32x16_bf16(bf16x8_ a, bf16x8_ b, f32x16_ c, int, int, int) {
  return mfma32(a, b, c, OP_MFMA32_BF16);
}

f32x4_ mfma_scale_f32_16x16x128_f8f6f4(i32x8_ a, i32x8_ b, f32x4_ c, int fa, int fb, int, int sa, int, int sb) {
  if (fa != 0 || fb != 0) {
    fprintf(stderr, "nvsim: only e4m3 operands are simulated\n");
    abort();
  }
  LaneIO& io = my_io();
  memcpy(io.a, &a, 32);
  memcpy(io.b, &b, 32);
  for (int r = 0; r < 4; ++r) io.acc[r] = c[r];
  io.sa = sa;
  io.sb = sb;
  wave_wait(OP_MFMA_F8);
  return f32x4_{io.res[0], io.res[1], io.res[2], io.res[3]};
}

int cvt_pk_fp8_f32(float a, float b, int old, bool hi) {
  const uint32_t pair = (uint32_t)f_to_e4m3(a) | ((uint32_t)f_to_e4m3(b) << 8);
  uint32_t w = (uint32_t)old;
  if (hi) w = (w & 0x0000ffffu) | (pair << 16);
  else w = (w & 0xffff0000u) | pair;
  return (int)w;
}

uint64_t shfl_xor_bits(uint64_t v, int mask, int width) {
  LaneIO& io = my_io();
  io.v = v;
  io.mask = mask;
  io.width = width;
  wave_wait(OP_SHFL);
  return io.vres;
}

int readfirstlane(int v) {
  LaneIO& io = my_io();
  io.v = (uint64_t)(uint32_t)v;
  wave_wait(OP_RFL);
  return (int)(uint32_t)io.vres;
}

void launch(dim3 grid, dim3 block, hipStream_t s, std::function<void()> body) {
  if (s && s->capturing) {
    s->rec->push_back([grid, block, body]() { launch(grid, block, nullptr, body); });
    return;
  }
  const int n = (int)(block.x * block.y * block.z);
  if (n <= 0 || n > 1024 || grid.x == 0 || grid.y == 0 || grid.z == 0) {
    fprintf(stderr, "nvsim: bad launch shape grid (%u,%u,%u) block (%u,%u,%u)\n", grid.x, grid.y, grid.z, block.x,
            block.y, block.z);
    abort();
  }
  const dim3 save_b = g_block_dim, save_g = g_grid_dim;
  g_block_dim = block;
  g_grid_dim = grid;
  for (unsigned z = 0; z < grid.z; ++z)
    for (unsigned y = 0; y < grid.y; ++y)
      for (unsigned x = 0; x < grid.x; ++x) {
        g_block = nvsim_uint3{x, y, z};
        run_block(body, n);
      }
  g_block_dim = save_b;
  g_grid_dim = save_g;
}

}  // namespace nvsim

// ------------------------------------------------------------------- runtime ----

namespace {
std::map<uintptr_t, size_t>& allocs() {
  static std::map<uintptr_t, size_t> m;
  return m;
}
void record_or_run(hipStream_t s, std::function<void()> op) {
  if (s && s->capturing) s->rec->push_back(std::move(op));
  else op();
}
}  // namespace

const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorInvalidValue: return "hipErrorInvalidValue";
    default: return "hipError(sim)";
  }
}
hipError_t hipMalloc(void** p, size_t bytes) {
  // uninitialised device memory: a fixed non-zero byte pattern, so that a kernel that
  // reads memory nobody wrote does not silently see zeros
  void* m = std::malloc(bytes ? bytes : 1);
  if (!m) return hipErrorOutOfMemory;
  std::memset(m, 0x7b, bytes);
  allocs()[reinterpret_cast<uintptr_t>(m)] = bytes;
  *p = m;
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipFree(void* p) {
  if (!p) return hipSuccess;
  auto it = allocs().find(reinterpret_cast<uintptr_t>(p));
  if (it == allocs().end()) return hipErrorInvalidValue;
  allocs().erase(it);
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  record_or_run(s, [=]() { std::memmove(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                             size_t height, hipMemcpyKind, hipStream_t s) {
  record_or_run(s, [=]() {
    for (size_t r = 0; r < height; ++r)
      std::memmove(static_cast<char*>(dst) + r * dpitch, static_cast<const char*>(src) + r * spitch, width);
  });
  return hipSuccess;
}
hipError_t hipMemset(void* p, int v, size_t bytes) {
  std::memset(p, v, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t s) {
  record_or_run(s, [=]() { std::memset(p, v, bytes); });
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  if (a == hipDeviceAttributeMaxSharedMemoryPerBlock) {
    *v = 160 * 1024;
    return hipSuccess;
  }
  return hipErrorInvalidValue;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new ihipStream_t;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s) return hipErrorInvalidValue;
  s->capturing = true;
  s->rec = new std::vector<std::function<void()>>;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capturing) return hipErrorInvalidValue;
  s->capturing = false;
  *g = new ihipGraph;
  (*g)->ops = std::move(*s->rec);
  delete s->rec;
  s->rec = nullptr;
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
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.001f;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, void*, void*, size_t) {
  *x = new hipGraphExec;
  (*x)->ops = g->ops;
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
// device-side statics are host statics in the simulation: the symbol's address is the array's
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  for (auto& op : x->ops) op();
  return hipSuccess;
}

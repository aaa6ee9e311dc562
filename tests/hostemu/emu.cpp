// Fiber scheduler and runtime calls of the host emulation (test
// infrastructure; see hip/hip_runtime.h).
#include "hip/hip_runtime.h"

#include <chrono>

// Switches stacks: saves the callee-saved registers on the current stack,
// stores its pointer in *save_sp and resumes the stack new_sp (x86-64).
extern "C" void emu_swap(void** save_sp, void* new_sp);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
)");

dim3 threadIdx, blockIdx, blockDim, gridDim;

namespace emu {
namespace {
enum St { RUN, WBLOCK, WWAVE, DONE };
struct Fiber {
  void* sp = nullptr;
  St st = RUN;
  char* stack = nullptr;
};
struct Blk {
  std::vector<Fiber> f;
  void* sched_sp = nullptr;
  const void* sched_bottom = nullptr;
  size_t sched_size = 0;
  int cur = 0, nt = 0;
  const std::function<void()>* body = nullptr;
  char* smem = nullptr;
  uint64_t xbits[1024];
  double xd[1024];
  double xb[1024];
};
Blk* g = nullptr;
bool g_capture = false;
std::vector<std::function<void()>>* g_rec = nullptr;
constexpr size_t STACK = 256 * 1024;

std::vector<char*> g_stacks;

void to_sched(Fiber& f) {
  emu_swap(&f.sp, g->sched_sp);
}
void fiber_main() {
  (*g->body)();
  g->f[g->cur].st = DONE;
  to_sched(g->f[g->cur]);
  std::abort();
}
void yield(St s) {
  Fiber& f = g->f[g->cur];
  f.st = s;
  to_sched(f);
}
}  // namespace

void block_barrier() { yield(WBLOCK); }
void wave_barrier() { yield(WWAVE); }
void* dyn_smem() { return g->smem; }
bool capturing() { return g_capture; }
void record(std::function<void()> f) { g_rec->push_back(std::move(f)); }

uint64_t ballot(bool p) {
  const int t = g->cur, base = t & ~63;
  g->xbits[t] = p ? 1 : 0;
  wave_barrier();
  uint64_t m = 0;
  for (int l = 0; l < 64 && base + l < g->nt; ++l)
    if (g->f[base + l].st != DONE && g->xbits[base + l]) m |= 1ull << l;
  wave_barrier();
  return m;
}
double shfl_d(double v, int src) {
  const int t = g->cur, base = t & ~63;
  g->xd[t] = v;
  wave_barrier();
  const double r = g->xd[base + src];
  wave_barrier();
  return r;
}
int shfl_i(int v, int src) { return int(shfl_d(double(v), src)); }

d4 mfma_f64_16x16x4(double a, double b, d4 c) {
  const int t = g->cur, base = t & ~63, l = t & 63;
  g->xd[t] = a;
  g->xb[t] = b;
  wave_barrier();
  d4 d = c;
  const int j = l % 16;
  for (int r = 0; r < 4; ++r) {
    const int i = l / 16 + 4 * r;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += g->xd[base + i + 16 * k] * g->xb[base + j + 16 * k];
    d[r] += s;
  }
  wave_barrier();
  return d;
}

// f32 16x16x4: same operand layout as the f64 form; lane l, register r of
// the result is row 4 (l / 16) + r, column l % 16 (the f64 form interleaves
// the rows, l / 16 + 4 r), as measured on gfx950.  Products and sums in
// float, k in order.
f4 mfma_f32_16x16x4(float a, float b, f4 c) {
  const int t = g->cur, base = t & ~63, l = t & 63;
  g->xd[t] = a;
  g->xb[t] = b;
  wave_barrier();
  f4 d = c;
  const int j = l % 16;
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * (l / 16) + r;
    float s = 0.0f;
    for (int k = 0; k < 4; ++k) s += float(g->xd[base + i + 16 * k]) * float(g->xb[base + j + 16 * k]);
    d[r] += s;
  }
  wave_barrier();
  return d;
}

static void run_block(int nt, size_t shmem, const std::function<void()>& body) {
  Blk b;
  b.nt = nt;
  b.body = &body;
  b.f.resize(nt);
  b.smem = shmem ? static_cast<char*>(std::malloc(shmem)) : nullptr;
  if (b.smem) std::memset(b.smem, 0xA5, shmem);
  Blk* prev = g;
  g = &b;
  while (int(g_stacks.size()) < nt) g_stacks.push_back(static_cast<char*>(std::malloc(STACK)));
  for (int i = 0; i < nt; ++i) {
    Fiber& f = b.f[i];
    f.stack = g_stacks[size_t(i)];
    uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + STACK) & ~uintptr_t(15);
    void** sp = reinterpret_cast<void**>(top - 64);
    for (int r = 0; r < 6; ++r) sp[r] = nullptr;
    sp[6] = reinterpret_cast<void*>(&fiber_main);
    sp[7] = nullptr;
    f.sp = sp;
  }
  while (true) {
    for (int i = 0; i < nt; ++i) {
      if (b.f[i].st != RUN) continue;
      b.cur = i;
      threadIdx = dim3(unsigned(i), 0, 0);
      emu_swap(&b.sched_sp, b.f[i].sp);
    }
    bool all_done = true, released = false;
    for (int i = 0; i < nt; ++i) all_done = all_done && b.f[i].st == DONE;
    if (all_done) break;
    // wave barriers: a wave whose live lanes all wait at a wave barrier
    for (int w0 = 0; w0 < nt; w0 += 64) {
      bool any = false, all = true;
      for (int l = w0; l < w0 + 64 && l < nt; ++l) {
        if (b.f[l].st == DONE) continue;
        any = true;
        if (b.f[l].st != WWAVE) all = false;
      }
      if (any && all) {
        for (int l = w0; l < w0 + 64 && l < nt; ++l)
          if (b.f[l].st == WWAVE) b.f[l].st = RUN;
        released = true;
      }
    }
    if (released) continue;
    bool allb = true;
    for (int i = 0; i < nt; ++i)
      if (b.f[i].st != DONE && b.f[i].st != WBLOCK) allb = false;
    if (allb) {
      for (int i = 0; i < nt; ++i)
        if (b.f[i].st == WBLOCK) b.f[i].st = RUN;
      continue;
    }
    std::fprintf(stderr, "emu: deadlock in block (%u,%u,%u) nt=%d\n", blockIdx.x, blockIdx.y, blockIdx.z, nt);
    for (int i = 0; i < nt; ++i) std::fprintf(stderr, " %d", int(b.f[i].st));
    std::fprintf(stderr, "\n");
    std::abort();
  }
  std::free(b.smem);
  g = prev;
}

void run_grid(dim3 gr, dim3 bl, size_t shmem, const std::function<void()>& body) {
  gridDim = gr;
  blockDim = bl;
  const int nt = int(bl.x * bl.y * bl.z);
  if (nt > 1024 || bl.y != 1 || bl.z != 1) {
    std::fprintf(stderr, "emu: unsupported block shape\n");
    std::abort();
  }
  for (unsigned z = 0; z < gr.z; ++z)
    for (unsigned y = 0; y < gr.y; ++y)
      for (unsigned x = 0; x < gr.x; ++x) {
        blockIdx = dim3(x, y, z);
        run_block(nt, shmem, body);
      }
}
}  // namespace emu

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emu error"; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (emu::capturing()) {
    emu::record([=]() { std::memmove(d, s, n); });
    return hipSuccess;
  }
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  if (emu::capturing()) {
    emu::record([=]() { std::memset(d, v, n); });
    return hipSuccess;
  }
  std::memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new int(1));
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<int*>(s);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new EmuEvent{0.0};
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }  // launches run in order
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->t = now_ms();
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = float(b->t - a->t);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned) {
  *p = std::malloc(n ? n : 1);
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  emu::g_capture = true;
  emu::g_rec = new std::vector<std::function<void()>>();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* gr) {
  emu::g_capture = false;
  *gr = emu::g_rec;
  emu::g_rec = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t gr, void*, char*, size_t) {
  *e = new std::vector<std::function<void()>>(*gr);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& f : *e) f();
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t gr) {
  delete gr;
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t spitch, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t) {
  auto f = [=]() {
    for (size_t r = 0; r < h; ++r)
      std::memmove(static_cast<char*>(d) + r * dp, static_cast<const char*>(s) + r * spitch, w);
  };
  if (emu::capturing())
    emu::record(f);
  else
    f();
  return hipSuccess;
}

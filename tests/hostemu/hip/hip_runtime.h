// Host emulation of the HIP subset the library uses (test infrastructure):
// every GPU thread of a block runs as a fiber on one OS thread, blocks run
// one after another, block and wave barriers and wave exchanges (ballot,
// shuffles, the FP64 16x16x4 matrix instruction) are emulated, and device
// memory is host memory.  Built with AddressSanitizer, it checks the kernels'
// memory accesses on the CPU.
#pragma once
#include <ucontext.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

// sine and cosine of pi x (device math functions that the host library
// does not provide)
inline void sincospi(double x, double* s, double* c) {
  *s = std::sin(M_PI * x);
  *c = std::cos(M_PI * x);
}
inline void sincospif(float x, float* s, float* c) {
  *s = std::sin(float(M_PI) * x);
  *c = std::cos(float(M_PI) * x);
}

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(x) __attribute__((aligned(x)))
#define __shared__ static

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern dim3 threadIdx, blockIdx, blockDim, gridDim;

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorLaunchFailure = 2 };
typedef void* hipStream_t;
struct EmuEvent { double t; };
typedef EmuEvent* hipEvent_t;
typedef std::vector<std::function<void()>>* hipGraph_t;
typedef std::vector<std::function<void()>>* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum { hipHostMallocDefault = 0 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };

namespace emu {
void block_barrier();
void wave_barrier();
uint64_t ballot(bool p);
double shfl_d(double v, int src);
int shfl_i(int v, int src);
void* dyn_smem();
void run_grid(dim3 g, dim3 b, size_t shmem, const std::function<void()>& body);
bool capturing();
void record(std::function<void()> f);
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
d4 mfma_f64_16x16x4(double a, double b, d4 c);
f4 mfma_f32_16x16x4(float a, float b, f4 c);

template <typename K>
struct Launch {
  K k;
  dim3 g, b;
  size_t sh;
  template <typename... A>
  void operator()(A... args) {
    K kk = k;
    dim3 gg = g, bb = b;
    size_t s = sh;
    auto f = [=]() { run_grid(gg, bb, s, [=]() { kk(args...); }); };
    if (capturing())
      record(f);
    else
      f();
  }
};
template <typename K>
Launch<K> launch(K k, dim3 g, dim3 b, size_t sh = 0, hipStream_t = nullptr) {
  return Launch<K>{k, g, b, sh};
}
}  // namespace emu

inline void __syncthreads() { emu::block_barrier(); }
inline void emu_amdgcn_wave_barrier() { emu::wave_barrier(); }
inline void emu_amdgcn_fence(int, const char*) {}
inline uint64_t __ballot(bool p) { return emu::ballot(p); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline int emu_amdgcn_readlane(int v, int l) { return emu::shfl_i(v, l & 63); }
// DPP lane moves of the controls the kernels use (quad_perm, row_shl/shr,
// row_mirror, row_half_mirror, row_bcast:15, row_bcast:31); lanes outside
// row_mask or with no valid source keep old (bound_ctrl false).
inline int emu_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int, bool bound_ctrl) {
  const int l = int(threadIdx.x) & 63, row = l >> 4, rl = l & 15;
  int s = -1;
  if (ctrl < 0x100) s = (l & ~3) + ((ctrl >> (2 * (l & 3))) & 3);
  else if (ctrl >= 0x101 && ctrl <= 0x10F) s = rl + (ctrl - 0x100) < 16 ? l + (ctrl - 0x100) : -1;
  else if (ctrl >= 0x111 && ctrl <= 0x11F) s = rl >= ctrl - 0x110 ? l - (ctrl - 0x110) : -1;
  else if (ctrl == 0x140) s = (l & ~15) + 15 - rl;
  else if (ctrl == 0x141) s = (l & ~7) + 7 - (l & 7);
  else if (ctrl == 0x142) s = row >= 1 ? (l & ~15) - 1 : -1;
  else if (ctrl == 0x143) s = row >= 2 ? 31 : -1;
  else std::abort();
  const int v = emu::shfl_i(src, s >= 0 ? s : l);  // every lane takes part
  if (!((row_mask >> row) & 1)) return old;
  if (s < 0) return bound_ctrl ? 0 : old;
  return v;
}
inline int emu_amdgcn_readfirstlane(int v) {
  const uint64_t m = emu::ballot(true);
  return emu::shfl_i(v, __builtin_ffsll((long long)m) - 1);
}
inline double __shfl_xor(double v, int m, int = 64) {
  return emu::shfl_d(v, (int(threadIdx.x) & 63) ^ m);
}
inline int __shfl_xor(int v, int m, int = 64) { return emu::shfl_i(v, (int(threadIdx.x) & 63) ^ m); }
inline double __shfl(double v, int src, int w = 64) {
  return emu::shfl_d(v, (int(threadIdx.x) & 63 & ~(w - 1)) + (src & (w - 1)));
}
inline int __shfl_up(int v, unsigned d, int w = 64) {
  const int l = int(threadIdx.x) & 63;
  return emu::shfl_i(v, (l & (w - 1)) >= int(d) ? l - int(d) : l);
}
inline int __shfl(int v, int src, int w = 64) {
  return emu::shfl_i(v, (int(threadIdx.x) & 63 & ~(w - 1)) + (src & (w - 1)));
}
inline float __uint_as_float(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
inline uint32_t __float_as_uint(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
inline int atomicOr(int* p, int v) { int o = *p; *p |= v; return o; }
inline int atomicMax(int* p, int v) { int o = *p; if (v > o) *p = v; return o; }
inline emu::d4 emu_amdgcn_mfma_f64_16x16x4f64(double a, double b, emu::d4 c, int, int, int) {
  return emu::mfma_f64_16x16x4(a, b, c);
}
inline emu::f4 emu_amdgcn_mfma_f32_16x16x4f32(float a, float b, emu::f4 c, int, int, int) {
  return emu::mfma_f32_16x16x4(a, b, c);
}

// ---- runtime API ----
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t = nullptr);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t = nullptr);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamCreateWithFlags(hipStream_t*, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipEventCreate(hipEvent_t*);
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t);
hipError_t hipHostMalloc(void**, size_t, unsigned = 0);
hipError_t hipMalloc(void**, size_t);
hipError_t hipFree(void*);
hipError_t hipGetDevice(int*);
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
hipError_t hipDeviceSynchronize();
hipError_t hipHostFree(void*);
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*);
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, char*, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t spitch, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t = nullptr);

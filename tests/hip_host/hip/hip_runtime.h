// Host build of the library's HIP sources for memory-safety checks (test infrastructure only:
// the product never loads it).  Emulates the HIP subset the sources use: every lane runs as a
// fiber and wavefront exchanges are resolved across the lanes of a wave (runtime.cpp).
#pragma once
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <type_traits>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __shared__ static thread_local
#define __constant__ static
#define __launch_bounds__(...)

using std::isfinite;
using std::isinf;
using std::isnan;

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef int hipMemcpyKind;
enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
struct EmuStream;
struct EmuEvent { int dummy; };
struct EmuGraph;
struct EmuGraphExec;
typedef EmuStream* hipStream_t;
typedef EmuEvent* hipEvent_t;
typedef EmuGraph* hipGraph_t;
typedef EmuGraphExec* hipGraphExec_t;
typedef void* hipGraphNode_t;
typedef int hipStreamCaptureMode;
enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1, hipStreamCaptureModeRelaxed = 2 };
typedef int hipGraphExecUpdateResult;
enum { hipGraphExecUpdateSuccess = 0, hipGraphExecUpdateError = 1 };
enum { hipStreamDefault = 0, hipStreamNonBlocking = 1 };
enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
enum { hipHostMallocDefault = 0 };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {
const dim3& tidx();
const dim3& bidx();
const dim3& bdim();
const dim3& gdim();
enum { OP_SHFL = 1, OP_SHFL_XOR, OP_SHFL_UP, OP_BALLOT, OP_ALL, OP_DPP, OP_READLANE, OP_SYNC, OP_WAVEBAR, OP_READFIRST };
uint64_t lane_op(int kind, uint64_t val, int a, int b, int c, int d, int e);
void launch(hipStream_t s, dim3 grid, dim3 block, std::function<void()> body);
template <class T> inline uint64_t bits(T v) { uint64_t u = 0; std::memcpy(&u, &v, sizeof(T)); return u; }
template <class T> inline T unbits(uint64_t u) { T v; std::memcpy(&v, &u, sizeof(T)); return v; }
}  // namespace emu

#define threadIdx (emu::tidx())
#define blockIdx (emu::bidx())
#define blockDim (emu::bdim())
#define gridDim (emu::gdim())

#define hipLaunchKernelGGL(kern, grid, block, shmem, stream, ...) \
  emu::launch((stream), dim3(grid), dim3(block), [=]() { kern(__VA_ARGS__); })

template <class T> inline T __shfl(T v, int src, int width = 64) { return emu::unbits<T>(emu::lane_op(emu::OP_SHFL, emu::bits(v), src, width, 0, 0, 0)); }
template <class T> inline T __shfl_xor(T v, int mask, int width = 64) { return emu::unbits<T>(emu::lane_op(emu::OP_SHFL_XOR, emu::bits(v), mask, width, 0, 0, 0)); }
template <class T> inline T __shfl_up(T v, unsigned delta, int width = 64) { return emu::unbits<T>(emu::lane_op(emu::OP_SHFL_UP, emu::bits(v), (int)delta, width, 0, 0, 0)); }
inline unsigned long long __ballot(int pred) { return emu::lane_op(emu::OP_BALLOT, pred ? 1 : 0, 0, 0, 0, 0, 0); }
inline int __all(int pred) { return (int)emu::lane_op(emu::OP_ALL, pred ? 1 : 0, 0, 0, 0, 0, 0); }
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound) {
  return (int)(uint32_t)emu::lane_op(emu::OP_DPP, ((uint64_t)(uint32_t)old << 32) | (uint32_t)src, ctrl, row_mask, bank_mask, bound ? 1 : 0, 0);
}
inline int __builtin_amdgcn_readlane(int v, int lane) { return (int)(uint32_t)emu::lane_op(emu::OP_READLANE, (uint32_t)v, lane, 0, 0, 0, 0); }
inline int __builtin_amdgcn_readfirstlane(int v) { return (int)(uint32_t)emu::lane_op(emu::OP_READFIRST, (uint32_t)v, 0, 0, 0, 0, 0); }
inline void __builtin_amdgcn_wave_barrier() { emu::lane_op(emu::OP_WAVEBAR, 0, 0, 0, 0, 0, 0); }
inline void __syncthreads() { emu::lane_op(emu::OP_SYNC, 0, 0, 0, 0, 0, 0); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline long long __double_as_longlong(double d) { long long v; std::memcpy(&v, &d, 8); return v; }
inline double __longlong_as_double(long long v) { double d; std::memcpy(&d, &v, 8); return d; }
inline int __float_as_int(float f) { int v; std::memcpy(&v, &f, 4); return v; }
inline float __int_as_float(int v) { float f; std::memcpy(&f, &v, 4); return f; }

// Blocks of a launch run on several host threads, so atomics are real ones.
template <class T> inline T atomicAdd(T* p, T v) {
  if constexpr (std::is_integral<T>::value) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
  } else {
    T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (!__atomic_compare_exchange_n(p, &o, o + v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
    return o;
  }
}
template <class T> inline T atomicMin(T* p, T v) {
  T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v < o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return o;
}
template <class T> inline T atomicMax(T* p, T v) {
  T o = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v > o && !__atomic_compare_exchange_n(p, &o, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return o;
}
template <class T> inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }

hipError_t hipMalloc(void** p, size_t n);
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
template <class T> inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) { return hipHostMalloc((void**)p, n, flags); }
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* n, char* log, size_t sz);
hipError_t hipGraphExecUpdate(hipGraphExec_t e, hipGraph_t g, hipGraphNode_t* n, hipGraphExecUpdateResult* r);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
